"""The interface system of one pairwise merge (Section 3.2; Section 6, eq. step1) from the oracle's
children, for the tests of the structured merges.

The children's Schur complements come from the oracle's recursive build; the blocks are cut from them and
from the assembled matrix exactly as the merge defines them:
  K_ii = [[S33, A34], [A43, S44]],  K_ie = [[S31, A32], [A41, S42]],  K_ee, K_ei likewise.
`pair` is the oracle's interface pair order (each P3 node followed by its five-point neighbour in P4).
"""
from __future__ import annotations

import numpy as np

from oracle import assemble
from oracle.grid import build_tree, box_ring
from oracle.nd import box_schur, merge_pair, interface_pair_order, _interior_to_union, _dense_block, lin


def root_merge_blocks(n, b=None, c=None, d=None, leaf=16, which="root"):
    """Blocks of the root merge (bottom + top halves) or, with which="bottom", of the SW + SE merge."""
    M = assemble(n, b, c, d)
    root = build_tree(n, leaf)
    keep = {}
    box_schur(M, n, root, keep)
    sw, se, nw, ne = root.children
    S_ = lambda bx: keep[(bx.x0, bx.x1, bx.y0, bx.y1)]
    if which == "bottom":
        box1, S1, box2, S2 = sw, S_(sw), se, S_(se)
    else:
        box1, S1 = merge_pair(M, n, sw, S_(sw), se, S_(se))
        box2, S2 = merge_pair(M, n, nw, S_(nw), ne, S_(ne))
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
    out = {
        "Kii": np.block([[S1[np.ix_(i3, i3)], blk(L3, L4)], [blk(L4, L3), S2[np.ix_(i4, i4)]]]),
        "Kie": np.block([[S1[np.ix_(i3, i1)], blk(L3, L2)], [blk(L4, L1), S2[np.ix_(i4, i2)]]]),
        "Kei": np.block([[S1[np.ix_(i1, i3)], blk(L1, L4)], [blk(L2, L3), S2[np.ix_(i2, i4)]]]),
        "Kee": np.block([[S1[np.ix_(i1, i1)], blk(L1, L2)], [blk(L2, L1), S2[np.ix_(i2, i2)]]]),
        "i1": len(P3),
        "pair": interface_pair_order(P3, P4),
    }
    return out
