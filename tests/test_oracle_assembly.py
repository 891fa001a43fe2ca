"""Pins for the oracle's assembly of the five-point system (paper Section 7)."""
import json
import os

import numpy as np
import pytest

from oracle import assemble, brute_dtn, ring_nodes
from oracle.assemble import ring_and_interior

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_derived_entries_n4():
    g = json.load(open(os.path.join(GOLD, "assemble_n4.json")))
    n = g["n"]
    b = np.zeros(n * n); c = np.zeros(n * n); d = np.zeros(n * n)
    k = 1 + n * 1
    b[k], c[k], d[k] = 3.0, -6.0, 9.0
    M = assemble(n, b, c, d).toarray()
    for r, col, v in g["entries_central"]:
        assert M[r, col] == pytest.approx(v, abs=1e-15), (r, col)
    Mp = assemble(n, b, c, d, conv="paper").toarray()
    for r, col, v in g["entries_paper_scale"]:
        assert Mp[r, col] == pytest.approx(v, abs=1e-15), (r, col)
    for r, cnt in g["row_nnz"].items():
        assert np.count_nonzero(M[int(r)]) == cnt


@pytest.mark.parametrize("n", [3, 4, 9, 16])
def test_row_sums_and_symmetry(n):
    rng = np.random.default_rng(n)
    h = 1.0 / (n - 1)
    d = rng.uniform(-3, 3, n * n)
    b = rng.uniform(-2, 2, n * n)
    c = rng.uniform(-2, 2, n * n)
    M = assemble(n, b, c, d)
    B, I = ring_and_interior(n)
    rs = np.asarray(M.sum(axis=1)).ravel()
    # interior rows: h^2 d_k (the differences of a constant vanish)
    assert np.allclose(rs[I], h * h * d[I], atol=1e-14)
    # ring rows (one-sided differences) and corner rows sum to zero
    assert np.allclose(rs[B], 0.0, atol=1e-15)
    Ms = assemble(n, None, None, d).toarray()
    assert np.array_equal(Ms, Ms.T)
    Mn = M.toarray()
    if n > 3:
        assert not np.allclose(Mn, Mn.T)


def test_laplace_is_grid_laplacian_minus_ring_links():
    n = 7
    M = assemble(n).toarray()
    ring = set(ring_nodes(n))
    L = np.zeros((n * n, n * n))
    for j in range(n):
        for i in range(n):
            for (a, bb) in ((i + 1, j), (i, j + 1)):
                if a < n and bb < n:
                    if (i, j) in ring and (a, bb) in ring:
                        continue
                    p, q = i + n * j, a + n * bb
                    L[p, q] -= 1; L[q, p] -= 1; L[p, p] += 1; L[q, q] += 1
    assert np.array_equal(M, L)


def test_n3_hand_dtn():
    g = json.load(open(os.path.join(GOLD, "dtn_n3.json")))
    mids = g["ring_midpoints"]
    for case in ("laplace", "helmholtz"):
        dv = g[case]["d"]
        T = brute_dtn(3, d=np.full(9, dv))
        E = np.zeros((8, 8))
        for a in mids:
            for bb in mids:
                E[a, bb] = g[case]["diag"] if a == bb else g[case]["offdiag"]
        assert np.allclose(T, E, atol=1e-14), case
