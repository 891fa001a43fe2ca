"""Pins for the oracle's DtN operator: brute force, closed forms and invariants.

Each test checks the oracle against something other than itself: a dense
Schur complement (Section 3.1), exact discrete solutions whose boundary flux
is known in closed form, discrete-sine separation of variables, or structural
invariants of Schur complements.
"""
import math

import numpy as np
import pytest

from oracle import (brute_dtn, build_tree, dst_dtn, nd_dtn, sparse_apply, trace_on_ring,
                    ring_nodes, leaf_schur, assemble, SingularError)
from oracle.grid import boxes_at_level, box_ring


def _rand_coeffs(n, rng, kind):
    if kind == "laplace":
        return None, None, None
    if kind == "cd":
        return rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    if kind == "helm":
        return None, None, np.full(n * n, -rng.uniform(10, 400))
    raise ValueError(kind)


@pytest.mark.parametrize("seed", range(12))
def test_nd_equals_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 41))
    leaf = int(rng.integers(4, 13))
    kind = ["laplace", "cd", "helm"][seed % 3]
    b, c, d = _rand_coeffs(n, rng, kind)
    T1 = brute_dtn(n, b, c, d)
    T2 = nd_dtn(n, b, c, d, leaf=leaf)
    # random Helmholtz shifts can sit close to a sub-box resonance, which amplifies
    # rounding by the local condition number; the other kinds are well conditioned
    rtol = 1e-9 if kind == "helm" else 1e-12
    assert np.abs(T1 - T2).max() <= rtol * max(1.0, np.abs(T1).max()), (n, leaf, kind)


@pytest.mark.parametrize("n", [5, 12, 23])
def test_brute_equals_sparse_solve(n):
    rng = np.random.default_rng(n)
    b, c, d = _rand_coeffs(n, rng, "cd")
    T = brute_dtn(n, b, c, d)
    G = rng.uniform(-1, 1, (4 * (n - 1), 5))
    Y = sparse_apply(n, G, b, c, d)
    assert np.allclose(T @ G, Y, atol=1e-12 * np.abs(Y).max())


def test_tree_independence():
    n = 64
    rng = np.random.default_rng(7)
    b, c, d = _rand_coeffs(n, rng, "cd")
    Ts = [nd_dtn(n, b, c, d, leaf=lf) for lf in (4, 8, 16, 33)]
    for T in Ts[1:]:
        assert np.abs(T - Ts[0]).max() <= 1e-12 * np.abs(Ts[0]).max()


@pytest.mark.parametrize("n", [17, 32, 45])
def test_constant_in_kernel_when_d_zero(n):
    rng = np.random.default_rng(n)
    b, c = rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n)
    T = nd_dtn(n, b, c, None, leaf=8)
    assert np.abs(T.sum(axis=1)).max() <= 1e-11 * np.abs(T).max()


def _laplace_exact(n):
    """Ring fluxes of discrete-harmonic polynomials (exact for the five-point stencil)."""
    h = 1.0 / (n - 1)
    ring = ring_nodes(n)
    out = {}
    side = []
    for (i, j) in ring:
        corner = (i in (0, n - 1)) and (j in (0, n - 1))
        if corner:
            side.append("C")
        elif j == 0:
            side.append("S")
        elif i == n - 1:
            side.append("E")
        elif j == n - 1:
            side.append("N")
        else:
            side.append("W")
    xs = np.array([p[0] * h for p in ring]); ys = np.array([p[1] * h for p in ring])
    f = {"S": h, "E": 2 - h, "N": -2 + h, "W": -h, "C": 0.0}
    out["x2-y2"] = (lambda x, y: x * x - y * y, np.array([f[s] for s in side]))
    e_xy = np.array([{"S": -x, "E": y, "N": x, "W": -y, "C": 0.0}[s] for s, x, y in zip(side, xs, ys)])
    out["xy"] = (lambda x, y: x * y, e_xy)
    out["x"] = (lambda x, y: x, np.array([{"E": 1.0, "W": -1.0}.get(s, 0.0) for s in side]))
    out["y"] = (lambda x, y: y, np.array([{"N": 1.0, "S": -1.0}.get(s, 0.0) for s in side]))
    return out


@pytest.mark.parametrize("n", [9, 33])
def test_laplace_polynomial_traces(n):
    T = nd_dtn(n, leaf=8)
    for name, (f, expect) in _laplace_exact(n).items():
        g = trace_on_ring(n, f)
        assert np.allclose(T @ g, expect, atol=1e-11), name


def test_laplace_polynomial_traces_sparse_large():
    n = 300
    ex = _laplace_exact(n)
    G = np.stack([trace_on_ring(n, f) for f, _ in ex.values()], axis=1)
    Y = sparse_apply(n, G)
    for q, (name, (_, expect)) in enumerate(ex.items()):
        assert np.allclose(Y[:, q], expect, atol=1e-9), name


@pytest.mark.parametrize("conv", ["central", "paper"])
@pytest.mark.parametrize("bc", [(3.0, -5.0), (-7.5, 2.0), (0.0, 9.0)])
def test_exponential_solution_constant_convection(conv, bc):
    """u = rho^i sigma^j solves the discrete convection-diffusion equation exactly (d = 0).

    With coefficient s = h/2 (centred) or h (paper scale) on the convection
    difference, rho = (1 + s b)/(1 - s b) and sigma = (1 + s c)/(1 - s c).
    """
    n = 21
    h = 1.0 / (n - 1)
    b0, c0 = bc
    s = h / 2 if conv == "central" else h
    rho, sig = (1 + s * b0) / (1 - s * b0), (1 + s * c0) / (1 - s * c0)
    u = lambda i, j: rho ** i * sig ** j
    ring = ring_nodes(n)
    g = np.array([u(i, j) for (i, j) in ring])
    expect = np.zeros(len(ring))
    for r, (i, j) in enumerate(ring):
        if (i in (0, n - 1)) and (j in (0, n - 1)):
            continue
        ii = 1 if i == 0 else (n - 2 if i == n - 1 else i)
        jj = 1 if j == 0 else (n - 2 if j == n - 1 else j)
        expect[r] = (u(i, j) - u(ii, jj)) / h
    bb = np.full(n * n, b0); cc = np.full(n * n, c0)
    T = nd_dtn(n, bb, cc, None, leaf=6, conv=conv)
    assert np.allclose(T @ g, expect, rtol=1e-10, atol=1e-10 * np.abs(expect).max())


@pytest.mark.parametrize("n,d", [(5, 0.0), (12, 0.0), (31, 0.0), (12, -150.0), (31, -900.0), (31, -3000.0)])
def test_dst_closed_form_equals_brute_force(n, d):
    T1 = brute_dtn(n, d=np.full(n * n, d))
    T2 = dst_dtn(n, d)
    assert np.abs(T1 - T2).max() <= 1e-11 * np.abs(T1).max()


def test_dst_closed_form_equals_sparse_solve_large():
    n = 257
    kappa = 12.3 * math.pi
    d = -kappa * kappa
    T = dst_dtn(n, d)
    rng = np.random.default_rng(5)
    G = rng.uniform(-1, 1, (4 * (n - 1), 6))
    Y = sparse_apply(n, G, None, None, np.full(n * n, d))
    assert np.linalg.norm(T @ G - Y) <= 1e-9 * np.linalg.norm(Y)


def test_symmetric_when_no_convection():
    n = 29
    rng = np.random.default_rng(3)
    d = rng.uniform(-50, 20, n * n)
    T = nd_dtn(n, None, None, d, leaf=8)
    assert np.abs(T - T.T).max() <= 1e-12 * np.abs(T).max()


def test_leaf_schur_laplace_row_sums_signs():
    """Laplace: box S'.1 counts each ring node's neighbours outside the box (zero on the global ring)."""
    n = 26
    M = assemble(n).tocsr()
    root = build_tree(n, 7)
    L = max(b.level for b in [root] + boxes_at_level(root, 1) + boxes_at_level(root, 2))
    for bx in boxes_at_level(root, 2):
        S = leaf_schur(M, n, bx)
        ring = box_ring(bx.x0, bx.x1, bx.y0, bx.y1)
        expect = []
        for (i, j) in ring:
            glob = i in (0, n - 1) or j in (0, n - 1)
            if glob:
                expect.append(0.0)
                continue
            out = sum(1 for (a, c_) in ((i + 1, j), (i - 1, j), (i, j + 1), (i, j - 1))
                      if not (bx.x0 <= a < bx.x1 and bx.y0 <= c_ < bx.y1))
            expect.append(float(out))
        assert np.allclose(S.sum(axis=1), expect, atol=1e-12)
        off = S - np.diag(np.diag(S))
        assert off.max() <= 1e-14
        assert np.abs(S - S.T).max() <= 1e-13


def test_singular_leaf_detected():
    """d = -mu/h^2 with mu a Dirichlet eigenvalue of a leaf's interior block makes it singular."""
    n, leaf = 17, 8
    h = 1.0 / (n - 1)
    root = build_tree(n, leaf)
    lf = boxes_at_level(root, max(1, 0))[0]
    while lf.children:
        lf = lf.children[0]
    m = lf.sx - 2
    assert lf.sx == lf.sy
    p = q = 1
    mu = 4 * math.sin(p * math.pi / (2 * (m + 1))) ** 2 + 4 * math.sin(q * math.pi / (2 * (m + 1))) ** 2
    d = np.full(n * n, -mu / (h * h))
    with pytest.raises(SingularError):
        nd_dtn(n, None, None, d, leaf=leaf)
    # slightly off the eigenvalue the build succeeds
    nd_dtn(n, None, None, d * (1 + 1e-3), leaf=leaf)
