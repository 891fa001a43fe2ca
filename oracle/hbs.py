"""Reference low-rank compression of off-diagonal blocks (oracle).

Section 6, Step 2 replaces the off-diagonal blocks S13 and S24 of the merge
formula by low-rank factorisations L R.  The paper defers the construction to
other work and runs it at a "local tolerance" (Section 7).  Reading used
here: a block is compressed by column-pivoted QR, truncated at the first
diagonal entry |r_kk| <= tol * |r_11|; the reference rank is that k.  Ranks of
a different rank-revealing method may differ by a few; reconstructions, not
factors, are compared.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def pivoted_qr_rank(A: np.ndarray, tol: float) -> int:
    """Rank of A at relative tolerance tol by column-pivoted QR."""
    A = np.asarray(A, dtype=np.float64)
    if A.size == 0:
        return 0
    R = sla.qr(A, mode="r", pivoting=True)[0]
    d = np.abs(np.diag(R))
    if d.size == 0 or d[0] == 0.0:
        return 0
    small = np.nonzero(d <= tol * d[0])[0]
    return int(small[0]) if small.size else int(d.size)


def low_rank(A: np.ndarray, tol: float):
    """(L, R) with A ~= L @ R, L = Q_k, R = (R P^T)[:k] from column-pivoted QR."""
    A = np.asarray(A, dtype=np.float64)
    Q, R, P = sla.qr(A, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    small = np.nonzero(d <= tol * (d[0] if d.size else 0.0))[0]
    k = int(small[0]) if small.size else int(d.size)
    Rk = np.zeros((k, A.shape[1]))
    Rk[:, P] = R[:k, :]
    return Q[:, :k], Rk


# ---------------------------------------------------------------------------
# Hierarchically block-separable (HBS) representation of a dense matrix, Section 4.
#
# Tree (Section 4.2.1): the index vector [0, M) is the root; an interval holding more than m indices
# is split into halves (floor / ceil), children listed left then right; levels count from the root.
# Factors (Section 4.3, def1-def6): a leaf tau holds D_tau = H(I_tau, I_tau); every node but the root
# holds U_tau and V_tau; every parent holds the sibling blocks of B_tau.  Section 4 defers the
# construction to other work; the reading used here: interpolative decompositions by column-pivoted
# QR at the local tolerance, from the leaves up.  A node's candidate rows R_tau (its indices at a
# leaf, its children's skeleton rows at a parent) are reduced by a row ID of the whole off-diagonal
# block row H(R_tau, complement of I_tau): H(R_tau, :) ~= U_tau H(J_tau, :) on those columns, J_tau
# the skeleton rows (pivots up to the first |r_kk| <= tol |r_11|), U_tau the interpolation matrix
# (identity on the skeleton rows).  Columns likewise (V_tau, skeleton columns J'_tau).  The sibling
# blocks of B_tau are then the submatrices H(J_s1, J'_s2) and H(J_s2, J'_s1), and the telescoping
# factorisation (tele1-tele3) holds to the tolerance.
# ---------------------------------------------------------------------------

def hbs_tree(M: int, m: int):
    """Nodes as dicts {lo, hi, level, children}; nodes[0] is the root, children after parents."""
    nodes = [{"lo": 0, "hi": M, "level": 0, "children": []}]
    q = 0
    while q < len(nodes):
        nd = nodes[q]
        if nd["hi"] - nd["lo"] > m:
            mid = nd["lo"] + (nd["hi"] - nd["lo"]) // 2
            for lo, hi in ((nd["lo"], mid), (mid, nd["hi"])):
                nd["children"].append(len(nodes))
                nodes.append({"lo": lo, "hi": hi, "level": nd["level"] + 1, "children": []})
        q += 1
    return nodes


def _row_id(A: np.ndarray, tol: float):
    """Row interpolative decomposition A ~= U A[J, :]: (J positions, U) by column-pivoted QR of A^T."""
    p = A.shape[0]
    if A.shape[1] == 0 or p == 0 or not np.any(A):
        return np.zeros(0, dtype=np.int64), np.zeros((p, 0))
    Q, R, P = sla.qr(A.T, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    small = np.nonzero(d <= tol * d[0])[0]
    k = int(small[0]) if small.size else int(d.size)
    X = sla.solve_triangular(R[:k, :k], R[:k, k:]) if k < p else np.zeros((k, 0))
    U = np.zeros((p, k))
    U[P[:k], :] = np.eye(k)
    U[P[k:], :] = X.T
    return np.asarray(P[:k], dtype=np.int64), U


def hbs_compress(H: np.ndarray, m: int, tol: float) -> dict:
    """HBS factors of a square H at local tolerance tol with leaves of at most m indices."""
    H = np.asarray(H, dtype=np.float64)
    M = H.shape[0]
    nodes = hbs_tree(M, m)
    depth = max(nd["level"] for nd in nodes)
    for lev in range(depth, 0, -1):
        for nd in nodes:
            if nd["level"] != lev:
                continue
            if nd["children"]:
                c1, c2 = (nodes[c] for c in nd["children"])
                rows = np.concatenate([c1["J"], c2["J"]])
                cols = np.concatenate([c1["Jc"], c2["Jc"]])
            else:
                rows = cols = np.arange(nd["lo"], nd["hi"])
                nd["D"] = H[nd["lo"]:nd["hi"], nd["lo"]:nd["hi"]].copy()
            out = np.r_[0:nd["lo"], nd["hi"]:M]
            jr, nd["U"] = _row_id(H[np.ix_(rows, out)], tol)
            jc, V = _row_id(H[np.ix_(out, cols)].T, tol)
            nd["V"] = V
            nd["J"], nd["Jc"] = rows[jr], cols[jc]
    if not nodes[0]["children"]:
        nodes[0]["D"] = H.copy()
    for nd in nodes:
        if nd["children"]:
            c1, c2 = (nodes[c] for c in nd["children"])
            nd["B12"] = H[np.ix_(c1["J"], c2["Jc"])]
            nd["B21"] = H[np.ix_(c2["J"], c1["Jc"])]
    return {"M": M, "m": m, "tol": tol, "nodes": nodes}


def hbs_apply(F: dict, X: np.ndarray) -> np.ndarray:
    """Y = H X through the telescoping factorisation: upward pass (V^T), sibling blocks, downward
    pass (U), leaf diagonal blocks."""
    nodes = F["nodes"]
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    X = X.reshape(F["M"], -1)
    xh, yh = {}, {}
    order = sorted(range(len(nodes)), key=lambda q: -nodes[q]["level"])
    for q in order:                                   # upward: leaves first
        nd = nodes[q]
        if q == 0:
            continue
        if nd["children"]:
            src = np.vstack([xh[c] for c in nd["children"]])
        else:
            src = X[nd["lo"]:nd["hi"]]
        xh[q] = nd["V"].T @ src
    for q, nd in enumerate(nodes):                    # sibling interactions
        if nd["children"]:
            c1, c2 = nd["children"]
            yh[c1] = nd["B12"] @ xh[c2]
            yh[c2] = nd["B21"] @ xh[c1]
    Y = np.zeros_like(X)
    for q in reversed(order):                         # downward: root side first
        nd = nodes[q]
        if q == 0:
            if not nd["children"]:
                Y[:] = nd["D"] @ X
            continue
        if nd["children"]:
            z = nd["U"] @ yh[q]
            c1, c2 = nd["children"]
            k1 = nodes[c1]["U"].shape[1]
            yh[c1] = yh[c1] + z[:k1]
            yh[c2] = yh[c2] + z[k1:]
        else:
            Y[nd["lo"]:nd["hi"]] = nd["D"] @ X[nd["lo"]:nd["hi"]] + nd["U"] @ yh[q]
    return Y[:, 0] if vec else Y


def hbs_dense(F: dict) -> np.ndarray:
    """The matrix an HBS representation stands for (its apply to the identity)."""
    return hbs_apply(F, np.eye(F["M"]))


def hbs_words(F: dict) -> int:
    """Stored numbers: leaf D blocks, every U and V, every sibling block (Table 2's memory / 8 bytes)."""
    w = 0
    for nd in F["nodes"]:
        for key in ("D", "U", "V", "B12", "B21"):
            if key in nd:
                w += nd[key].size
    return w


def hbs_ranks(F: dict) -> list:
    """Largest row or column rank per level (index 0 = root, which has none)."""
    depth = max(nd["level"] for nd in F["nodes"])
    out = [0] * (depth + 1)
    for nd in F["nodes"]:
        if "U" in nd:
            out[nd["level"]] = max(out[nd["level"]], nd["U"].shape[1], nd["V"].shape[1])
    return out


# ---------------------------------------------------------------------------
# Inversion of an HBS matrix (Section 5.1, Algorithm 1) and the application of the inverse
# (Algorithm 2), in the paper's notation.  Algorithm 1 needs square, well-conditioned V^* D~^{-1} U
# at every node.  The paper leaves the construction of the HBS factors to other work; with separate
# row and column skeletons the two ranks differ, and forcing them equal leaves V^* D~^{-1} U with
# condition numbers up to ~1e10 on the convection problems of Section 7.1, so hbs_compress_square takes
# one skeleton set per node from its block row and block column together.
# Reading of Algorithm 2's garbles: its downward pass and leaf step use y^_tau (printed x^_tau and q^_tau).
# ---------------------------------------------------------------------------

def hbs_compress_square(H: np.ndarray, m: int, tol: float) -> dict:
    """HBS factors with one skeleton set and one interpolation matrix per node for its block row and
    block column together (so U = V and the ranks are equal, as Algorithm 1 needs): the row ID at tol of
    [H(R, out), H(out, R)^T] for the node's candidates R (a leaf's indices, else its children's
    skeletons) and the indices `out` outside the node."""
    H = np.asarray(H, dtype=np.float64)
    M = H.shape[0]
    nodes = hbs_tree(M, m)
    depth = max(nd["level"] for nd in nodes)
    for lev in range(depth, 0, -1):
        for nd in nodes:
            if nd["level"] != lev:
                continue
            if nd["children"]:
                c1, c2 = (nodes[c] for c in nd["children"])
                rows = np.concatenate([c1["J"], c2["J"]])
            else:
                rows = np.arange(nd["lo"], nd["hi"])
                nd["D"] = H[nd["lo"]:nd["hi"], nd["lo"]:nd["hi"]].copy()
            out = np.r_[0:nd["lo"], nd["hi"]:M]
            j, W = _row_id(np.hstack([H[np.ix_(rows, out)], H[np.ix_(out, rows)].T]), tol)
            nd["U"], nd["V"] = W, W.copy()
            nd["J"] = nd["Jc"] = rows[j]
    if not nodes[0]["children"]:
        nodes[0]["D"] = H.copy()
    for nd in nodes:
        if nd["children"]:
            c1, c2 = (nodes[c] for c in nd["children"])
            nd["B12"] = H[np.ix_(c1["J"], c2["Jc"])]
            nd["B21"] = H[np.ix_(c2["J"], c1["Jc"])]
    return {"M": M, "m": m, "tol": tol, "nodes": nodes}


def hbs_invert(F: dict) -> dict:
    """Algorithm 1: factors {E, F*, G} of H^{-1} from the HBS factors {U, V, D, B} of H, levels finer to
    coarser; at the root G_1 = [[D^_2, B_23], [B_32, D^_3]]^{-1}."""
    nodes = F["nodes"]
    depth = max(nd["level"] for nd in nodes)
    inv = [dict() for _ in nodes]
    for lev in range(depth, 0, -1):
        for q, nd in enumerate(nodes):
            if nd["level"] != lev:
                continue
            if not nd["children"]:
                Dt = nd["D"]
            else:
                s1, s2 = nd["children"]
                Dt = np.block([[inv[s1]["Dhat"], nd["B12"]], [nd["B21"], inv[s2]["Dhat"]]])
            Dinv = np.linalg.inv(Dt)
            U, V = nd["U"], nd["V"]
            Dhat = np.linalg.inv(V.T @ Dinv @ U)
            inv[q]["Dhat"] = Dhat
            inv[q]["E"] = Dinv @ U @ Dhat
            inv[q]["Fs"] = Dhat @ V.T @ Dinv                      # F^*
            inv[q]["G"] = Dinv - Dinv @ U @ Dhat @ V.T @ Dinv
    root = nodes[0]
    if root["children"]:
        s1, s2 = root["children"]
        inv[0]["G"] = np.linalg.inv(np.block([[inv[s1]["Dhat"], root["B12"]], [root["B21"], inv[s2]["Dhat"]]]))
    else:
        inv[0]["G"] = np.linalg.inv(root["D"])
    return {"M": F["M"], "nodes": nodes, "inv": inv}


def hbs_inverse_apply(Fi: dict, X: np.ndarray) -> np.ndarray:
    """Algorithm 2: y = H^{-1} x from Algorithm 1's factors (upward pass with F^*, root block G_1,
    downward pass with E and G, leaves)."""
    nodes, inv = Fi["nodes"], Fi["inv"]
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    X = X.reshape(Fi["M"], -1)
    root = nodes[0]
    if not root["children"]:
        Y = inv[0]["G"] @ X
        return Y[:, 0] if vec else Y
    depth = max(nd["level"] for nd in nodes)
    xh, yh = {}, {}
    for q, nd in enumerate(nodes):                            # leaves
        if q and not nd["children"]:
            xh[q] = inv[q]["Fs"] @ X[nd["lo"]:nd["hi"]]
    for lev in range(depth, 0, -1):                           # parents, finer to coarser
        for q, nd in enumerate(nodes):
            if q and nd["level"] == lev and nd["children"]:
                xh[q] = inv[q]["Fs"] @ np.vstack([xh[c] for c in nd["children"]])
    s1, s2 = root["children"]
    z = inv[0]["G"] @ np.vstack([xh[s1], xh[s2]])
    k1 = xh[s1].shape[0]
    yh[s1], yh[s2] = z[:k1], z[k1:]
    for lev in range(1, depth):                               # parents, coarser to finer
        for q, nd in enumerate(nodes):
            if q and nd["level"] == lev and nd["children"]:
                c1, c2 = nd["children"]
                z = inv[q]["E"] @ yh[q] + inv[q]["G"] @ np.vstack([xh[c1], xh[c2]])
                k1 = xh[c1].shape[0]
                yh[c1], yh[c2] = z[:k1], z[k1:]
    Y = np.zeros_like(X)
    for q, nd in enumerate(nodes):                            # leaves
        if q and not nd["children"]:
            Y[nd["lo"]:nd["hi"]] = inv[q]["E"] @ yh[q] + inv[q]["G"] @ X[nd["lo"]:nd["hi"]]
    return Y[:, 0] if vec else Y
