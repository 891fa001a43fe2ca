"""GPU tests of the inverse HBS factors (Section 5.1, Algorithms 1 and 2) through the C ABI.

With the R2 ring rows the built T is S'/h for the Schur complement S' of the whole grid's five-point
matrix onto the ring, so T^{-1} = h G with G = S'^{-1} the paper's solution operator (Section 7).  The
exact value of G r comes from the oracle's sparse solve of the full system with r on the ring
(Section 7.1's protocol); e1 uses a unit vector of random direction, e2 a smooth one.  The factors are
not unique, so only their applies are compared: with the oracle's G, with the oracle's own
Algorithm 1 / 2 on the oracle's operator, and through the residual T (T^{-1} R) - R with the dense T.
The convection problems (diffusion-convection I, III, IV of Section 7.1) are the ones whose inverse
needs one skeleton set per node for its block row and column together.
"""
import numpy as np
import pytest

import workloads as W
from oracle import nd_dtn, solution_apply
from oracle.hbs import hbs_compress_square, hbs_invert, hbs_inverse_apply

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


def _coeffs(kind, n):
    if kind in W.PAPER_PROBLEMS:
        P = W.paper_problem(kind, n)
        return P.b, P.c, P.d
    rng = np.random.default_rng(n + 3)
    return rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)


def _rel(a, b):
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


@pytest.mark.parametrize("n,leaf,kind,tol,bound", [
    (257, 64, "laplace", 1e-10, 1e-7), (257, 64, "helmholtz1", 1e-10, 1e-7),
    (257, 64, "diffconv1", 1e-10, 1e-7), (257, 64, "diffconv3", 1e-10, 1e-7), (257, 64, "diffconv4", 1e-10, 1e-7),
    (129, 32, "varcoef", 1e-10, 1e-7), (33, 8, "varcoef", 1e-11, 1e-8)])
def test_inverse_vs_solution_operator(dtn, n, leaf, kind, tol, bound):
    b, c, d = _coeffs(kind, n)
    op = dtn.build(n, b, c, d, leaf=16 if n > 64 else 8, ring_rows=dtn.RING_R2)
    T = op.dense()
    info = op.hbs_invert(tol, leaf)
    assert info["bytes"] > 0 and info["levels"] >= 1
    R = W.error_vectors(n)
    h = 1.0 / (n - 1)
    Y = op.apply_hbs_inverse_device(_dev(R)).cpu().numpy()
    G_ref = solution_apply(n, R, b, c, d)
    e = _rel(Y / h, G_ref)
    res = _rel(T @ Y, R)
    print(f"n={n} {kind} tol={tol}: e1 {e[0]:.3e} e2 {e[1]:.3e} residual {res.max():.3e} "
          f"ranks {info['max_rank']} MB {info['bytes'] / 1e6:.3f}", flush=True)
    assert np.all(e <= bound), e
    assert np.all(res <= 100 * tol), res
    # the oracle's Algorithm 1 / 2 on the oracle's operator, same tree and tolerance
    Tref = nd_dtn(n, b, c, d, leaf=16 if n > 64 else 8, ring_rows="R2")
    Yo = hbs_inverse_apply(hbs_invert(hbs_compress_square(Tref, leaf, tol)), R)
    assert np.all(_rel(Y, Yo) <= bound), _rel(Y, Yo)
    op.free()


def test_inverse_root_leaf(dtn):
    """A ring of at most `leaf` positions: the root is a leaf and T^{-1} is its one inverted block."""
    n = 9
    b, c, d = _coeffs("varcoef", n)
    op = dtn.build(n, b, c, d, leaf=4, ring_rows=dtn.RING_R2)
    T = op.dense()
    info = op.hbs_invert(1e-12, 64)
    assert info["levels"] == 0 and info["launches"] == 1
    R = W.error_vectors(n)
    Y = op.apply_hbs_inverse_device(_dev(R)).cpu().numpy()
    ref = np.linalg.solve(T, R)
    assert np.abs(Y - ref).max() <= 1e-12 * np.abs(ref).max()
    G_ref = solution_apply(n, R, b, c, d)
    assert np.all(_rel(Y * (n - 1), G_ref) <= 1e-11)
    op.free()


def test_inverse_many_columns_and_repeat(dtn):
    """k = 130 columns (several 32-column chunks and a ragged tail), an inverse rebuilt at another
    tolerance replaces the first, and the result is bitwise repeatable."""
    n = 129
    b, c, d = _coeffs("varcoef", n)
    op = dtn.build(n, b, c, d, leaf=16, ring_rows=dtn.RING_R2)
    T = op.dense()
    op.hbs_invert(1e-6, 32)
    info = op.hbs_invert(1e-10, 48)
    assert info["tol"] == 1e-10 and info["leaf"] == 48
    X = np.random.default_rng(3).uniform(-1, 1, (op.nb, 130))
    Xd = _dev(X)
    Y1 = op.apply_hbs_inverse_device(Xd).cpu().numpy()
    Y2 = op.apply_hbs_inverse_device(Xd).cpu().numpy()
    assert np.array_equal(Y1, Y2)
    assert np.all(_rel(T @ Y1, X) <= 1e-8)
    op.free()


def test_inverse_errors(dtn):
    n = 33
    op = dtn.build(n, leaf=8, ring_rows=dtn.RING_R2)
    R = _dev(W.error_vectors(n))
    with pytest.raises(dtn.DtnError):
        op.apply_hbs_inverse_device(R)          # not inverted yet
    with pytest.raises(dtn.DtnError):
        op.hbs_invert(0.0, 32)                  # tol must be > 0
    with pytest.raises(dtn.DtnError):
        op.hbs_invert(1e-8, 4)                  # leaf out of [8, 64]
    op.hbs_compress(1e-8, 16, drop_dense=True)
    with pytest.raises(dtn.DtnError):
        op.hbs_invert(1e-8, 16)                 # the dense T is gone
    op.free()
