"""Nested-dissection build of the boundary operator (oracle).

Follows the paper's Section 3.3 in order:

1. Build the quadtree (Section 2; see `grid.build_tree`).
2. For every leaf box P, form the Schur complement of its local matrix onto
   its ring (Section 3.1): S = A_bb - A_bi A_ii^{-1} A_ib, where the interior
   block A_ii is banded and is solved as such (Section 3.4 uses the band to
   bound the leaf cost).
3. Going up the tree, the Schur complement of a box is obtained from those
   of its four children by three pairwise merges (Section 3.3, step 3).  A
   pairwise merge of boxes w and e (Section 3.2) splits the ring of w into
   P1 (on the ring of the union) and P3 (interior to the union), and the ring
   of e into P2 and P4 likewise, and evaluates

       S = [S11 A12; A21 S22] - [S13 A14; A23 S24] [S33 A34; A43 S44]^{-1} [S31 A32; A41 S42]

   where the A blocks are the couplings of the original matrix between the
   node sets.  All A blocks are taken from the assembled matrix, even those
   that vanish for the five-point stencil (A14, A23, A32, A41).
4. At the root the Schur complement of the whole domain is available;
   T = S / h is the discrete DtN operator.

Structured merges (Section 6, Step 1; option kii_tol > 0): at the merges whose children's rings both
reach kii_min_ring nodes, X = K_ii^{-1} K_ie is formed through the HBS form of K_ii (Algorithms 1 and 2
of Section 5.1, `hbs.py`) instead of the LU, with K_ii taken in the interface pair order (each P3 node
followed by its five-point neighbour in P4): in the plain order [P3; P4] the anti-diagonal coupling A34 is
a full-rank off-diagonal block, in the pair order every off-diagonal block of the binary tree has low rank.

Readings: children are merged as (SW+SE), (NW+NE), then (bottom+top); every
box ring is counter-clockwise from its SW corner; the merged rows/columns
[P1; P2] are reordered to the union's ring order.  Factorisations use LU with
partial pivoting (LAPACK gbtrf/getrf).  A factorisation whose smallest pivot
magnitude is below PIVOT_RTOL times the largest matrix entry raises
SingularError.
"""
from __future__ import annotations

from typing import Dict, Optional, Tuple

import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack

from .assemble import assemble
from .grid import Box, box_interior, box_ring, build_tree, lin
from .hbs import hbs_compress_square, hbs_invert, hbs_inverse_apply

PIVOT_RTOL = 1e-11
KII_LEAF = 64          # HBS leaf size of a structured merge's interface block


class SingularError(ArithmeticError):
    """A leaf interior block or a merge interface block is numerically singular."""


def _check_pivots(diagU: np.ndarray, scale: float, what: str):
    if diagU.size == 0:
        return
    if not np.all(np.isfinite(diagU)) or np.min(np.abs(diagU)) <= PIVOT_RTOL * scale:
        raise SingularError(f"singular {what}: min |pivot| = {np.min(np.abs(diagU)):.3e}, scale {scale:.3e}")


def _dense_block(M, rows_lin: np.ndarray, cols_lin: np.ndarray) -> np.ndarray:
    if rows_lin.size == 0 or cols_lin.size == 0:
        return np.zeros((rows_lin.size, cols_lin.size))
    return M[rows_lin][:, cols_lin].toarray()


def leaf_schur(M, n: int, box: Box) -> np.ndarray:
    """Schur complement of a leaf's local matrix onto its ring (Section 3.1), banded interior solve."""
    ring = box_ring(box.x0, box.x1, box.y0, box.y1)
    inter = box_interior(box.x0, box.x1, box.y0, box.y1)
    rl, il = lin(n, ring), lin(n, inter)
    Abb = _dense_block(M, rl, rl)
    if il.size == 0:
        return Abb
    Abi = _dense_block(M, rl, il)
    Aib = _dense_block(M, il, rl)
    Aii = _dense_block(M, il, il)
    # interior ordered row by row: bandwidth = interior width
    w = box.sx - 2
    m = il.size
    kl = ku = min(w, m - 1)
    ab = np.zeros((2 * kl + ku + 1, m))
    for dgl in range(-kl, ku + 1):               # band storage for gbtrf: ab[kl+ku+i-j, j] = A[i, j]
        if dgl >= 0:
            vals = np.diagonal(Aii, dgl)         # A[j-dgl, j]
            ab[kl + ku - dgl, dgl:] = vals
        else:
            vals = np.diagonal(Aii, dgl)         # A[j+|dgl|, j]
            ab[kl + ku - dgl, :m + dgl] = vals
    lub, piv, info = lapack.dgbtrf(ab, kl, ku)
    if info < 0:
        raise RuntimeError("dgbtrf argument error")
    _check_pivots(lub[kl + ku, :], np.max(np.abs(Aii)), "leaf interior block")
    X, info = lapack.dgbtrs(lub, kl, ku, Aib, piv)
    if info != 0:
        raise RuntimeError("dgbtrs failed")
    return Abb - Abi @ X


def _interior_to_union(p: Tuple[int, int], n: int, U: Tuple[int, int, int, int]) -> bool:
    x0, x1, y0, y1 = U
    i, j = p
    for (a, b) in ((i + 1, j), (i - 1, j), (i, j + 1), (i, j - 1)):
        if not (0 <= a < n and 0 <= b < n):
            return False
        if not (x0 <= a < x1 and y0 <= b < y1):
            return False
    return True


def interface_pair_order(P3, P4) -> np.ndarray:
    """Positions in [P3; P4] of the interface pair order: each P3 node, then its unused grid neighbour in
    P4 (the node across the shared edge)."""
    at4 = {p: k for k, p in enumerate(P4)}
    used = set()
    src = []
    for r, (i, j) in enumerate(P3):
        hit = None
        for q in ((i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1)):
            k = at4.get(q)
            if k is not None and k not in used:
                hit = k
                break
        if hit is None:
            raise ValueError("interface node without a partner across the shared edge")
        used.add(hit)
        src += [r, len(P3) + hit]
    if len(src) != len(P3) + len(P4):
        raise ValueError("interface lines of different lengths")
    return np.array(src, dtype=np.int64)


def merge_pair(M, n: int, box1: Box, S1: np.ndarray, box2: Box, S2: np.ndarray, kii_tol: float = 0.0):
    """Pairwise merge of Section 3.2; returns (union box, S of the union in its ring order).  kii_tol > 0:
    K_ii^{-1} K_ie through the HBS form of K_ii in the interface pair order (Section 6, Step 1)."""
    U = (min(box1.x0, box2.x0), max(box1.x1, box2.x1), min(box1.y0, box2.y0), max(box1.y1, box2.y1))
    ring1 = box_ring(box1.x0, box1.x1, box1.y0, box1.y1)
    ring2 = box_ring(box2.x0, box2.x1, box2.y0, box2.y1)
    in1 = np.array([_interior_to_union(p, n, U) for p in ring1])
    in2 = np.array([_interior_to_union(p, n, U) for p in ring2])
    i1 = np.nonzero(~in1)[0]   # P1
    i3 = np.nonzero(in1)[0]    # P3
    i2 = np.nonzero(~in2)[0]   # P2
    i4 = np.nonzero(in2)[0]    # P4
    P1 = [ring1[t] for t in i1]
    P3 = [ring1[t] for t in i3]
    P2 = [ring2[t] for t in i2]
    P4 = [ring2[t] for t in i4]
    L1, L2, L3, L4 = lin(n, P1), lin(n, P2), lin(n, P3), lin(n, P4)

    S11, S13 = S1[np.ix_(i1, i1)], S1[np.ix_(i1, i3)]
    S31, S33 = S1[np.ix_(i3, i1)], S1[np.ix_(i3, i3)]
    S22, S24 = S2[np.ix_(i2, i2)], S2[np.ix_(i2, i4)]
    S42, S44 = S2[np.ix_(i4, i2)], S2[np.ix_(i4, i4)]
    A12, A21 = _dense_block(M, L1, L2), _dense_block(M, L2, L1)
    A14, A23 = _dense_block(M, L1, L4), _dense_block(M, L2, L3)
    A32, A41 = _dense_block(M, L3, L2), _dense_block(M, L4, L1)
    A34, A43 = _dense_block(M, L3, L4), _dense_block(M, L4, L3)

    Tee = np.block([[S11, A12], [A21, S22]])
    Tei = np.block([[S13, A14], [A23, S24]])
    Tie = np.block([[S31, A32], [A41, S42]])
    Tii = np.block([[S33, A34], [A43, S44]])
    if Tii.shape[0] > 0 and kii_tol > 0.0:
        src = interface_pair_order(P3, P4)
        Xp = hbs_inverse_apply(hbs_invert(hbs_compress_square(Tii[np.ix_(src, src)], KII_LEAF, kii_tol)), Tie[src])
        X = np.empty_like(Xp)
        X[src] = Xp
        S = Tee - Tei @ X
    elif Tii.shape[0] > 0:
        lu, piv = sla.lu_factor(Tii, check_finite=False)
        _check_pivots(np.diag(lu), np.max(np.abs(Tii)), "merge interface block")
        S = Tee - Tei @ sla.lu_solve((lu, piv), Tie, check_finite=False)
    else:
        S = Tee
    ext = P1 + P2
    pos = {p: t for t, p in enumerate(ext)}
    parent_ring = box_ring(*U)
    perm = np.array([pos[p] for p in parent_ring])
    ub = Box(U[0], U[1], U[2], U[3], min(box1.level, box2.level))
    return ub, S[np.ix_(perm, perm)]


def box_schur(M, n: int, box: Box, keep: Optional[Dict] = None, kii_tol: float = 0.0,
              kii_min_ring: int = 1000) -> np.ndarray:
    """Schur complement of `box` onto its ring by the recursive build (Section 3.3); kii_tol > 0 makes
    the merges whose children's rings both have >= kii_min_ring nodes structured (Section 6, Step 1)."""
    if not box.children:
        S = leaf_schur(M, n, box)
    else:
        sw, se, nw, ne = box.children
        Ssw = box_schur(M, n, sw, keep, kii_tol, kii_min_ring)
        Sse = box_schur(M, n, se, keep, kii_tol, kii_min_ring)
        Snw = box_schur(M, n, nw, keep, kii_tol, kii_min_ring)
        Sne = box_schur(M, n, ne, keep, kii_tol, kii_min_ring)
        tol_of = lambda S1, S2: kii_tol if min(len(S1), len(S2)) >= kii_min_ring else 0.0
        bot, Sbot = merge_pair(M, n, sw, Ssw, se, Sse, tol_of(Ssw, Sse))
        del Ssw, Sse
        top, Stop = merge_pair(M, n, nw, Snw, ne, Sne, tol_of(Snw, Sne))
        del Snw, Sne
        _, S = merge_pair(M, n, bot, Sbot, top, Stop, tol_of(Sbot, Stop))
    if keep is not None:
        keep[(box.x0, box.x1, box.y0, box.y1)] = S
    return S


def nd_dtn(n: int, b=None, c=None, d=None, leaf: int = 8, conv: str = "central",
           M=None, keep: Optional[Dict] = None, ring_rows: str = "R1", form: str = "pde",
           kii_tol: float = 0.0, kii_min_ring: int = 1000) -> np.ndarray:
    """T = S_root / h by nested dissection; rows/cols in global ring order (ring-row reading and
    coefficient form as in `assemble`; structured merges as in `box_schur`)."""
    if M is None:
        M = assemble(n, b, c, d, conv, ring_rows, form)
    M = M.tocsr()
    root = build_tree(n, leaf)
    S = box_schur(M, n, root, keep, kii_tol, kii_min_ring)
    return S / (1.0 / (n - 1))
