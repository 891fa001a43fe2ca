"""Assembly of the five-point system (oracle).

Section 7 of the paper discretises -Lap u + b u_x + c u_y + d u = 0 on the unit
square with the five-point stencil on an n x n grid, h = 1/(n-1): at an
interior node k with neighbours k_e, k_w, k_n, k_s,

    (1/h^2) [4 u(k) - u(k_n) - u(k_s) - u(k_w) - u(k_e)]
      + b(k) D_x u(k) + c(k) D_y u(k) + d(k) u(k).

Readings (the paper is silent or inconsistent here):
* Convection.  The paper prints (1/h) b(k) [u(k_e) - u(k_w)], a centred
  difference without the factor 1/2.  By default the centred derivative
  [u(k_e) - u(k_w)] / (2h) is used (consistent with b u_x); conv="paper"
  selects the printed 1/h scale.
* Boundary rows.  The sought output is the normal derivative on the
  boundary (Section 1.1).  The boundary ring is kept as a set of unknowns
  whose rows are the one-sided outward difference u(b) - u(b_in), b_in the
  inward neighbour; the four corners, which no stencil touches, get zero
  rows.  The Schur complement of the whole matrix onto the ring, divided by
  h, is then the discrete DtN map T: (T g)(b) = (g(b) - u(b_in)) / h for the
  discrete solution u with u = g on the ring.

The matrix returned is M' = h^2 * (interior operator) with the ring rows
above; it is symmetric exactly when b = c = 0.

Ring-row readings (`ring_rows`).  Section 3.1 takes the outermost ring of
*unknown* nodes as the boundary set, with the full equilibrium equation in
its rows; Section 1.1 asks for the normal derivative on the boundary.  The
three readings differ only in the ring rows:
* "R1" (default) - the one-sided differences above (a DtN map: T 1 = 0 when
  d = 0);
* "R2" - every ring node, corners included, keeps the full h^2-scaled
  five-point row of the grid with the couplings to nodes outside the grid
  dropped (the ring taken as the outermost ring of unknowns of Section 3.1,
  with zero data beyond it), using the coefficients at the ring node;
* "R3" - the R1 rows plus the ring-cycle graph Laplacian: each ring node
  also couples with weight 1 to its two neighbours along the ring (the
  Laplacian of the whole grid graph, Kron-reduced onto the ring, when
  b = c = d = 0).

Network form (`form="network"`, Section 7.1's random Laplacians): the grid is a
network of links with conductances, and an interior node's equation says its
potential is the conductance-weighted average of its four neighbours' -
sum over its links of sigma (u_k - u_l) + h^2 d_k u_k = 0 - with the
conductance of link (i,j)-(i+1,j) in b[i + n j] and of (i,j)-(i,j+1) in
c[i + n j].  Unit conductances give the Laplace rows.  A ring node's R1 row is
then the current through its inward link, sigma (u(b) - u(b_in)) (so the
operator is symmetric and annihilates constants); ring rows as R1 or R3.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import scipy.sparse as sp


def _field(n: int, f: Optional[np.ndarray]) -> np.ndarray:
    if f is None:
        return np.zeros(n * n)
    f = np.asarray(f, dtype=np.float64).reshape(-1)
    if f.size != n * n:
        raise ValueError("coefficient field must have n*n entries")
    return f


def assemble(n: int, b=None, c=None, d=None, conv: str = "central", ring_rows: str = "R1",
             form: str = "pde") -> sp.csr_matrix:
    """Return M' (n^2 x n^2, CSR) for the grid problem; node (i, j) has index i + n*j."""
    if n < 3:
        raise ValueError("n must be >= 3")
    h = 1.0 / (n - 1)
    bf, cf, df = _field(n, b), _field(n, c), _field(n, d)
    if conv == "central":
        cs = h / 2.0
    elif conv == "paper":
        cs = h
    else:
        raise ValueError("conv must be 'central' or 'paper'")

    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ii, jj = ii.reshape(-1), jj.reshape(-1)
    k = ii + n * jj
    on_x = (ii == 0) | (ii == n - 1)
    on_y = (jj == 0) | (jj == n - 1)
    interior = ~(on_x | on_y)
    ring = (on_x ^ on_y)                  # boundary ring minus the four corners (zero rows)

    rows, cols, vals = [], [], []
    # interior node: h^2 times the five-point operator
    ki = k[interior]
    rows += [ki] * 5
    cols += [ki, ki + 1, ki - 1, ki + n, ki - n]
    if form == "network":
        se, sw, sn, ss = bf[ki], bf[ki - 1], cf[ki], cf[ki - n]   # the node's four link conductances
        vals += [se + sw + sn + ss + h * h * df[ki], -se, -sw, -sn, -ss]
    elif form == "pde":
        vals += [4.0 + h * h * df[ki],
                 -1.0 + cs * bf[ki],          # east
                 -1.0 - cs * bf[ki],          # west
                 -1.0 + cs * cf[ki],          # north
                 -1.0 - cs * cf[ki]]          # south
    else:
        raise ValueError("form must be 'pde' or 'network'")
    if form == "network" and ring_rows == "R2":
        raise ValueError("the R2 ring rows are defined for the PDE form only")
    if ring_rows not in ("R1", "R2", "R3"):
        raise ValueError("ring_rows must be 'R1', 'R2' or 'R3'")
    if ring_rows == "R2":
        # every ring node (corners included): the five-point row, neighbours outside the grid dropped
        kb, ib, jb = k[on_x | on_y], ii[on_x | on_y], jj[on_x | on_y]
        rows.append(kb)
        cols.append(kb)
        vals.append(4.0 + h * h * df[kb])
        for di, dj, coef in ((1, 0, -1.0 + cs * bf[kb]), (-1, 0, -1.0 - cs * bf[kb]),
                             (0, 1, -1.0 + cs * cf[kb]), (0, -1, -1.0 - cs * cf[kb])):
            inside = (ib + di >= 0) & (ib + di <= n - 1) & (jb + dj >= 0) & (jb + dj <= n - 1)
            rows.append(kb[inside])
            cols.append(kb[inside] + di + n * dj)
            vals.append(coef[inside])
    else:
        # ring node (not a corner): one-sided difference towards the inward neighbour
        kr, ir, jr = k[ring], ii[ring], jj[ring]
        iin = np.where(ir == 0, 1, np.where(ir == n - 1, n - 2, ir))
        jin = np.where(jr == 0, 1, np.where(jr == n - 1, n - 2, jr))
        kin = iin + n * jin
        # network form: the current sigma (u(b) - u(b_in)) through the ring node's inward link, whose
        # conductance sits at the link's lower-left node (b for horizontal links, c for vertical ones)
        w = np.ones(kr.size)
        if form == "network":
            w = np.where(jr == 0, cf[kr], np.where(jr == n - 1, cf[np.minimum(kin, kr)],
                         np.where(ir == 0, bf[kr], bf[np.minimum(kin, kr)])))
        rows += [kr, kr]
        cols += [kr, kin]
        vals += [w, -w]
    if ring_rows == "R3":
        # ring-cycle Laplacian: weight-1 links between consecutive ring nodes (corners included)
        from .grid import ring_nodes, lin
        B = lin(n, ring_nodes(n))
        nxt = np.roll(B, -1)
        rows += [B, B, nxt, nxt]
        cols += [B, nxt, nxt, B]
        vals += [np.ones(B.size), -np.ones(B.size), np.ones(B.size), -np.ones(B.size)]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))
    M.sum_duplicates()
    return M


def ring_and_interior(n: int):
    """Linear indices of the boundary ring (counter-clockwise from (0,0)) and of the interior."""
    from .grid import ring_nodes, lin
    B = lin(n, ring_nodes(n))
    I = np.array([i + n * j for j in range(1, n - 1) for i in range(1, n - 1)], dtype=np.int64)
    return B, I
