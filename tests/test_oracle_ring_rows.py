"""Oracle pins for the three ring-row readings (Section 3.1's boundary set versus Section 1.1's normal
derivative).

R1 keeps one-sided differences on the ring, R2 the full five-point rows of the ring nodes (outside
couplings dropped), R3 the R1 rows plus the ring-cycle Laplacian.  Pinned here by things the
definitions fix, independently of the oracle's own nested dissection:
* three different eliminations (dense Schur complement, sparse LU of the interior, nested
  dissection) agree for every reading;
* R3 - R1 is exactly the cycle Laplacian over h (the interior rows and the inward couplings are
  common to both readings, so the Schur complements differ by the ring-ring block only);
* Laplace under R2: every row of S' sums to the number of the node's grid neighbours outside the
  grid (1 on an edge, 2 at a corner), because the full five-point row of a constant sums to that
  number and the interior rows of a constant sum to zero;
* without convection the R2 operator is symmetric, and for b = c = 0 it differs from R1 by the
  ring-ring block of the five-point rows (diagonal 3 + h^2 d on edges, 4 + h^2 d at corners, -1
  between ring neighbours), an identity written out here entry by entry.
"""
import numpy as np
import pytest

from oracle import brute_dtn, nd_dtn, sparse_apply, ring_nodes


def cycle_laplacian(nb):
    L = 2.0 * np.eye(nb)
    for r in range(nb):
        L[r, (r + 1) % nb] = L[r, (r - 1) % nb] = -1.0
    return L


@pytest.mark.parametrize("n,leaf,seed", [(9, 4, 1), (17, 8, 2), (24, 6, 3)])
@pytest.mark.parametrize("rows", ["R1", "R2", "R3"])
def test_three_eliminations_agree(n, leaf, seed, rows):
    rng = np.random.default_rng(seed)
    b, c, d = rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    Tb = brute_dtn(n, b, c, d, ring_rows=rows)
    Tn = nd_dtn(n, b, c, d, leaf=leaf, ring_rows=rows)
    G = rng.uniform(-1, 1, (4 * (n - 1), 3))
    Ys = sparse_apply(n, G, b, c, d, ring_rows=rows)
    scale = np.abs(Tb).max()
    assert np.abs(Tb - Tn).max() <= 1e-13 * scale
    assert np.abs(Ys - Tb @ G).max() <= 1e-13 * np.abs(Ys).max()


def test_r3_is_r1_plus_cycle_laplacian():
    n = 21
    rng = np.random.default_rng(5)
    b, c, d = rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(-30, 16, n * n)
    h = 1.0 / (n - 1)
    T1 = brute_dtn(n, b, c, d)
    T3 = brute_dtn(n, b, c, d, ring_rows="R3")
    assert np.abs(T3 - T1 - cycle_laplacian(4 * (n - 1)) / h).max() <= 1e-12 * np.abs(T3).max()


def test_laplace_r2_row_sums_count_outside_neighbours():
    n = 20
    h = 1.0 / (n - 1)
    S2 = brute_dtn(n, ring_rows="R2") * h
    rs = S2.sum(axis=1)
    expect = np.array([2.0 if (i in (0, n - 1) and j in (0, n - 1)) else 1.0 for (i, j) in ring_nodes(n)])
    assert np.abs(rs - expect).max() <= 1e-12


def test_r2_without_convection_is_r1_plus_ring_block():
    n = 19
    rng = np.random.default_rng(8)
    d = rng.uniform(-40, 20, n * n)
    h = 1.0 / (n - 1)
    T1 = brute_dtn(n, None, None, d)
    T2 = brute_dtn(n, None, None, d, ring_rows="R2")
    ring = ring_nodes(n)
    nb = len(ring)
    dM = np.zeros((nb, nb))
    for r, (i, j) in enumerate(ring):
        corner = i in (0, n - 1) and j in (0, n - 1)
        dM[r, r] = (4.0 if corner else 3.0) + h * h * d[i + n * j]
        dM[r, (r + 1) % nb] = dM[r, (r - 1) % nb] = -1.0
    assert np.abs(T2 - T1 - dM / h).max() <= 1e-12 * np.abs(T2).max()
    assert np.abs(T2 - T2.T).max() <= 1e-12 * np.abs(T2).max()


def test_bad_reading_rejected():
    with pytest.raises(ValueError):
        brute_dtn(5, ring_rows="R4")
