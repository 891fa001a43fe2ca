"""Body loads (oracle; test infrastructure): the operator F of Section 7.3 that maps loads at a fixed set
of interior nodes to the boundary fluxes, v = T g + F f_hat.

With the ring rows of the R1 reading (the flux rows of `assemble`), the load f_hat_j at interior node k_j
enters the interior equations as h^2 f_hat_j (the operator M' is h^2-scaled), so for g = 0 the interior
potential is u_I = M'_II^{-1} h^2 P f_hat (P places the loads) and the flux rows give
    v = (M'_BI u_I) / h,   i.e.   F = h M'_BI M'_II^{-1} P.
`body_operator` evaluates that definition with one sparse LU of M'_II.  `body_nested` follows the
nested dissection of Section 3.3 instead: every box carries, besides its Schur complement, the condensed
right-hand sides of the loads inside it (the leaf's update and, at each pairwise merge, the update of
Section 3.2: [f1; f2] - K_ei K_ii^{-1} [f3; f4]), and at the root F = -(condensed right-hand side) / h.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .assemble import assemble, ring_and_interior
from .grid import Box, box_interior, box_ring, build_tree, lin
from .nd import _dense_block, _interior_to_union


def body_operator(n: int, nodes, b=None, c=None, d=None, conv: str = "central", form: str = "pde") -> np.ndarray:
    """F (nb x len(nodes)) for loads at the interior nodes (i, j) in `nodes`, by a sparse solve."""
    nodes = [tuple(map(int, p)) for p in nodes]
    for i, j in nodes:
        if not (0 < i < n - 1 and 0 < j < n - 1):
            raise ValueError("body nodes must be interior nodes")
    M = assemble(n, b, c, d, conv, "R1", form).tocsc()
    B, I = ring_and_interior(n)
    h = 1.0 / (n - 1)
    pos = {k: t for t, k in enumerate(I)}
    P = np.zeros((len(I), len(nodes)))
    for q, (i, j) in enumerate(nodes):
        P[pos[i + n * j], q] = h * h
    lu = spla.splu(M[I][:, I].tocsc())
    U = lu.solve(P)
    return (M[B][:, I] @ U) / h


def _leaf_rhs(M, n: int, box: Box, loads: Dict[Tuple[int, int], int], nq: int) -> np.ndarray:
    """Condensed right-hand sides on the ring of a leaf box (ring x nq): r_ring - A_ri A_ii^{-1} r_int."""
    ring = box_ring(box.x0, box.x1, box.y0, box.y1)
    inner = box_interior(box.x0, box.x1, box.y0, box.y1)
    h2 = 1.0 / (n - 1) ** 2
    R = np.zeros((len(ring), nq))
    Ri = np.zeros((len(inner), nq))
    for t, p in enumerate(ring):
        if p in loads:
            R[t, loads[p]] = h2
    for t, p in enumerate(inner):
        if p in loads:
            Ri[t, loads[p]] = h2
    if inner and np.any(Ri):
        Lr, Li = lin(n, ring), lin(n, inner)
        Aii = _dense_block(M, Li, Li)
        Ari = _dense_block(M, Lr, Li)
        R -= Ari @ sla.solve(Aii, Ri)
    return R


def _merge_rhs(M, n: int, box1: Box, S1, R1, box2: Box, S2, R2):
    """Pairwise merge of Section 3.2 carrying the condensed right-hand sides; returns (box, S, R) in the
    union's ring order."""
    U = (min(box1.x0, box2.x0), max(box1.x1, box2.x1), min(box1.y0, box2.y0), max(box1.y1, box2.y1))
    ring1 = box_ring(box1.x0, box1.x1, box1.y0, box1.y1)
    ring2 = box_ring(box2.x0, box2.x1, box2.y0, box2.y1)
    in1 = np.array([_interior_to_union(p, n, U) for p in ring1])
    in2 = np.array([_interior_to_union(p, n, U) for p in ring2])
    i1, i3 = np.nonzero(~in1)[0], np.nonzero(in1)[0]
    i2, i4 = np.nonzero(~in2)[0], np.nonzero(in2)[0]
    P1, P3 = [ring1[t] for t in i1], [ring1[t] for t in i3]
    P2, P4 = [ring2[t] for t in i2], [ring2[t] for t in i4]
    L1, L2, L3, L4 = lin(n, P1), lin(n, P2), lin(n, P3), lin(n, P4)
    blk = lambda a, b_: _dense_block(M, a, b_)
    Tee = np.block([[S1[np.ix_(i1, i1)], blk(L1, L2)], [blk(L2, L1), S2[np.ix_(i2, i2)]]])
    Tei = np.block([[S1[np.ix_(i1, i3)], blk(L1, L4)], [blk(L2, L3), S2[np.ix_(i2, i4)]]])
    Tie = np.block([[S1[np.ix_(i3, i1)], blk(L3, L2)], [blk(L4, L1), S2[np.ix_(i4, i2)]]])
    Tii = np.block([[S1[np.ix_(i3, i3)], blk(L3, L4)], [blk(L4, L3), S2[np.ix_(i4, i4)]]])
    Re = np.vstack([R1[i1], R2[i2]])
    Ri = np.vstack([R1[i3], R2[i4]])
    if Tii.shape[0] > 0:
        lu = sla.lu_factor(Tii, check_finite=False)
        S = Tee - Tei @ sla.lu_solve(lu, Tie, check_finite=False)
        R = Re - Tei @ sla.lu_solve(lu, Ri, check_finite=False)
    else:
        S, R = Tee, Re
    pos = {p: t for t, p in enumerate(P1 + P2)}
    perm = np.array([pos[p] for p in box_ring(*U)])
    return Box(U[0], U[1], U[2], U[3], min(box1.level, box2.level)), S[np.ix_(perm, perm)], R[perm]


def body_nested(n: int, nodes, b=None, c=None, d=None, leaf: int = 8, conv: str = "central",
                form: str = "pde") -> Tuple[np.ndarray, np.ndarray]:
    """(T, F) by nested dissection with the loads' right-hand sides carried through every merge."""
    from .nd import leaf_schur
    M = assemble(n, b, c, d, conv, "R1", form).tocsr()
    loads = {tuple(map(int, p)): q for q, p in enumerate(nodes)}
    nq = len(loads)

    def rec(box: Box):
        if not box.children:
            return leaf_schur(M, n, box), _leaf_rhs(M, n, box, loads, nq)
        sw, se, nw, ne = box.children
        (S_sw, R_sw), (S_se, R_se) = rec(sw), rec(se)
        (S_nw, R_nw), (S_ne, R_ne) = rec(nw), rec(ne)
        bot, S_b, R_b = _merge_rhs(M, n, sw, S_sw, R_sw, se, S_se, R_se)
        top, S_t, R_t = _merge_rhs(M, n, nw, S_nw, R_nw, ne, S_ne, R_ne)
        _, S, R = _merge_rhs(M, n, bot, S_b, R_b, top, S_t, R_t)
        return S, R

    h = 1.0 / (n - 1)
    S, R = rec(build_tree(n, leaf))
    return S / h, -R / h
