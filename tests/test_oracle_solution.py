"""Pins of the oracle's solution operator G = S'^{-1} (Section 7; the e1 / e2 errors of Section 7.1).

* Constant d, b = c = 0 with the R2 ring rows: M' is the h^2-scaled Dirichlet five-point matrix of the
  whole n x n grid, K (x) I + I (x) K + h^2 d with K = tridiag(-1, 2, -1), diagonalised by the discrete
  sine transform; its inverse applied to r_hat, restricted to the ring, must equal solution_apply.
* Any coefficients, tiny grids: G R equals the inverse of the dense Schur complement (itself pinned
  against brute force) applied to R, and h G R equals T^{-1} R for T of the R2 reading.
* The error vectors: unit norms, ring coordinates on the boundary.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.assemble import ring_and_interior


def _dst_solve(n, d, rhat):
    """(K (x) I + I (x) K + h^2 d I)^{-1} rhat by the 2-D sine transform (node (i, j) at i + n j)."""
    h = 1.0 / (n - 1)
    p = np.arange(1, n + 1)
    S = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(p, p) * math.pi / (n + 1))   # orthogonal, symmetric
    lam = 4.0 * np.sin(p * math.pi / (2.0 * (n + 1))) ** 2
    R = rhat.reshape(n, n)                  # [j, i]
    Rh = S @ R @ S
    X = Rh / (lam[:, None] + lam[None, :] + h * h * d)
    return (S @ X @ S).reshape(-1)


@pytest.mark.parametrize("n,d", [(5, 0.0), (17, 0.0), (33, -100.0), (65, -4005.0), (40, 37.0)])
def test_solution_apply_matches_sine_transform(n, d):
    R = W.error_vectors(n, seed=11)
    B = np.asarray(oracle.ring_nodes(n))
    lin = B[:, 0] + n * B[:, 1]
    got = oracle.solution_apply(n, R, d=np.full(n * n, d))
    for k in range(R.shape[1]):
        rhat = np.zeros(n * n)
        rhat[lin] = R[:, k]
        ref = _dst_solve(n, d, rhat)[lin]
        assert np.linalg.norm(got[:, k] - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("n", [4, 7, 12])
def test_solution_apply_is_inverse_schur(n):
    rng = np.random.default_rng(n)
    b = rng.uniform(-30, 30, n * n)
    c = rng.uniform(-30, 30, n * n)
    d = rng.uniform(-5, 5, n * n)
    R = rng.standard_normal((4 * (n - 1), 3))
    M = oracle.assemble(n, b, c, d, ring_rows="R2").toarray()
    B, I = ring_and_interior(n)
    S = oracle.schur_complement(M, B, I)
    got = oracle.solution_apply(n, R, b, c, d)
    assert np.abs(got - np.linalg.solve(S, R)).max() <= 1e-11 * np.abs(got).max()
    h = 1.0 / (n - 1)
    T = oracle.brute_dtn(n, b, c, d, ring_rows="R2")
    assert np.abs(h * got - np.linalg.solve(T, R)).max() <= 1e-11 * np.abs(h * got).max()


def test_error_vectors():
    for n in (3, 9, 64):
        R = W.error_vectors(n)
        assert R.shape == (4 * (n - 1), 2) and R.flags.f_contiguous
        assert np.allclose(np.linalg.norm(R, axis=0), 1.0)
        x, y = W.ring_xy(n)
        on = (np.isclose(x, 0) | np.isclose(x, 1) | np.isclose(y, 0) | np.isclose(y, 1))
        assert on.all()
