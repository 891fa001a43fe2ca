"""Pins for the oracle's low-rank reference (`oracle.hbs`) and for the global ring order.

Compression (Section 4.1, block-separable rank; Section 6 Step 2; Section 7's local
tolerance): matrices with a prescribed singular spectrum U diag(s) V^T whose gap straddles
the tolerance have a rank fixed by the mathematics, and an exact low-rank product must be
recovered to rounding.  A transposed permutation, a dropped pivot or an off-by-one in the
truncation each fail one of these.

Ring order (Section 3.1's boundary nodes; the ABI's row order): ring index r = s (n - 1) + t,
t = 0 .. n - 2, with side s = 0 south (t, 0), 1 east (n - 1, t), 2 north (n - 1 - t, n - 1),
3 west (0, n - 1 - t), written out here node by node for n = 3, 4, 5.
"""
import json
import os

import numpy as np
import pytest

from oracle import ring_nodes, ring_index_of
from oracle.hbs import low_rank, pivoted_qr_rank

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _spectrum_matrix(m, n, s, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, len(s))))
    V, _ = np.linalg.qr(rng.standard_normal((n, len(s))))
    return (U * np.asarray(s)) @ V.T


@pytest.mark.parametrize("m,n,r,seed", [(60, 40, 7, 1), (40, 60, 12, 2), (90, 90, 30, 3), (25, 25, 1, 4)])
def test_pivoted_qr_rank_at_a_spectral_gap(m, n, r, seed):
    # r singular values in [1e-3, 1], the rest at 1e-14: the gap straddles tol = 1e-8 by far more
    # than the O(sqrt(n)) factor by which pivoted-QR diagonals can differ from singular values
    k = min(m, n)
    big = np.logspace(0, -3, r)
    s = np.concatenate([big, np.full(k - r, 1e-14)])
    A = _spectrum_matrix(m, n, s, seed)
    assert pivoted_qr_rank(A, 1e-8) == r
    # a tolerance above the whole upper part of the spectrum leaves only the leading column
    assert pivoted_qr_rank(A, 0.999) <= 2
    # with no small singular values and a tolerance below the smallest, the rank is full
    B = _spectrum_matrix(m, n, np.logspace(0, -2, k), seed + 10)
    assert pivoted_qr_rank(B, 1e-6) == k


def test_pivoted_qr_rank_special_cases():
    assert pivoted_qr_rank(np.zeros((5, 4)), 1e-10) == 0
    assert pivoted_qr_rank(np.zeros((0, 4)), 1e-10) == 0
    u, v = np.arange(1.0, 8.0), np.linspace(-1.0, 2.0, 5)
    assert pivoted_qr_rank(np.outer(u, v), 1e-12) == 1
    assert pivoted_qr_rank(np.eye(6), 1e-12) == 6
    # a diagonal matrix: pivoted QR sorts the diagonal, so the rank at tol counts entries > tol * max
    D = np.diag([1.0, 1e-3, 1e-9, 1e-12, 0.5])
    assert pivoted_qr_rank(D, 1e-11) == 4
    assert pivoted_qr_rank(D, 1e-8) == 3
    assert pivoted_qr_rank(D, 1e-2) == 2


@pytest.mark.parametrize("m,n,r,seed", [(50, 30, 5, 5), (30, 70, 9, 6), (80, 80, 20, 7)])
def test_low_rank_recovers_exact_low_rank_products(m, n, r, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    L, R = low_rank(A, 1e-12)
    assert L.shape == (m, r) and R.shape == (r, n)
    assert np.allclose(L.T @ L, np.eye(r), atol=1e-13)
    assert np.linalg.norm(A - L @ R) <= 1e-13 * np.linalg.norm(A)


@pytest.mark.parametrize("tol", [1e-4, 1e-8, 1e-11])
def test_low_rank_error_at_the_tolerance_scale(tol):
    # geometric spectrum: the truncated factorisation's error is of the size of the first
    # discarded singular value, between tol/10 and 10 tol times the norm (pivoted QR is
    # rank-revealing up to modest factors)
    m, n = 70, 50
    s = np.logspace(0, -15, n)
    A = _spectrum_matrix(m, n, s, 11)
    L, R = low_rank(A, tol)
    k = L.shape[1]
    assert k == pivoted_qr_rank(A, tol)
    err = np.linalg.norm(A - L @ R, 2)
    assert tol / 100 <= err <= 100 * tol, (k, err)
    # the rank is within a few of the number of singular values above tol
    assert abs(k - int(np.sum(s > tol))) <= 3


def _ring_by_formula(n):
    out = []
    for s in range(4):
        for t in range(n - 1):
            out.append([(t, 0), (n - 1, t), (n - 1 - t, n - 1), (0, n - 1 - t)][s])
    return out


def test_ring_order_written_out():
    assert ring_nodes(3) == [(0, 0), (1, 0), (2, 0), (2, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    assert ring_nodes(4) == [(0, 0), (1, 0), (2, 0), (3, 0), (3, 1), (3, 2), (3, 3), (2, 3), (1, 3),
                             (0, 3), (0, 2), (0, 1)]
    assert ring_nodes(5) == [(0, 0), (1, 0), (2, 0), (3, 0), (4, 0), (4, 1), (4, 2), (4, 3), (4, 4),
                             (3, 4), (2, 4), (1, 4), (0, 4), (0, 3), (0, 2), (0, 1)]


@pytest.mark.parametrize("n", [3, 4, 5, 6, 17, 64])
def test_ring_order_formula(n):
    ring = ring_nodes(n)
    assert ring == _ring_by_formula(n)
    assert len(ring) == 4 * (n - 1) == len(set(ring))
    # corners at r = 0, n-1, 2(n-1), 3(n-1)
    assert [ring[q * (n - 1)] for q in range(4)] == [(0, 0), (n - 1, 0), (n - 1, n - 1), (0, n - 1)]
    # every step is to a grid neighbour, and the last node neighbours the first (a closed cycle)
    for a, b in zip(ring, ring[1:] + ring[:1]):
        assert abs(a[0] - b[0]) + abs(a[1] - b[1]) == 1
    idx = ring_index_of(n)
    assert all(idx[p] == r for r, p in enumerate(ring))


def test_ring_order_matches_the_golden_text():
    g = json.load(open(os.path.join(GOLD, "dtn_n3.json")))
    assert "[(0,0),(1,0),(2,0),(2,1),(2,2),(1,2),(0,2),(0,1)]" in g["source"].replace(" ", "")
    assert [ring_nodes(3)[q] for q in g["ring_midpoints"]] == [(1, 0), (2, 1), (1, 2), (0, 1)]
