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
