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
