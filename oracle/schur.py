"""Schur complement onto the boundary ring, by direct definition (oracle).

Section 3.1: partitioning the unknowns of a set P into interior nodes i and
boundary nodes b, eliminating u_i gives S = A_bb - A_bi A_ii^{-1} A_ib.  For
the whole grid, with the boundary ring as b (see `assemble`), S' / h is the
discrete DtN map T.

* `schur_complement` - dense S for an explicit partition (tiny sizes).
* `brute_dtn`        - T for the whole grid via one dense solve (n <= ~48).
* `sparse_apply`     - Y = T G via one sparse LU of the interior block, i.e.
                       solving the full system for the interior potential
                       with the ring values prescribed, then taking the ring
                       rows: (T g)(b) = (M'_BB g + M'_BI u_I)(b) / h.
* `solution_apply`   - X = G R for the solution operator G = S'^{-1} of
                       Section 7 (the inverse of the whole domain's Schur
                       complement), through one sparse LU of the full system:
                       M' x = r_hat with r_hat = r on the ring and 0 inside
                       gives x on the ring = S'^{-1} r (block elimination of the
                       interior unknowns), which is how Section 7.1 obtains the
                       exact value of G r for its errors e1 and e2.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import assemble, ring_and_interior


def schur_complement(A: np.ndarray, bidx, iidx) -> np.ndarray:
    """S = A_bb - A_bi A_ii^{-1} A_ib for a dense A (Section 3.1)."""
    A = np.asarray(A, dtype=np.float64)
    bidx = np.asarray(bidx)
    iidx = np.asarray(iidx)
    Abb = A[np.ix_(bidx, bidx)]
    if iidx.size == 0:
        return Abb.copy()
    Abi = A[np.ix_(bidx, iidx)]
    Aib = A[np.ix_(iidx, bidx)]
    Aii = A[np.ix_(iidx, iidx)]
    return Abb - Abi @ np.linalg.solve(Aii, Aib)


def brute_dtn(n: int, b=None, c=None, d=None, conv: str = "central", ring_rows: str = "R1",
              form: str = "pde") -> np.ndarray:
    """Dense T = S'/h of the whole grid (ring order counter-clockwise from (0,0))."""
    if n > 64:
        raise ValueError("brute_dtn is for tiny grids (n <= 64)")
    M = assemble(n, b, c, d, conv, ring_rows, form).toarray()
    B, I = ring_and_interior(n)
    h = 1.0 / (n - 1)
    return schur_complement(M, B, I) / h


def sparse_apply(n: int, G: np.ndarray, b=None, c=None, d=None, conv: str = "central",
                 M: sp.csr_matrix = None, ring_rows: str = "R1", form: str = "pde") -> np.ndarray:
    """Y = T G through one sparse direct solve of the interior system."""
    if M is None:
        M = assemble(n, b, c, d, conv, ring_rows, form)
    B, I = ring_and_interior(n)
    h = 1.0 / (n - 1)
    G = np.asarray(G, dtype=np.float64)
    if G.ndim == 1:
        G = G[:, None]
    M = M.tocsr()
    MII = M[I][:, I].tocsc()
    MIB = M[I][:, B]
    MBB = M[B][:, B]
    MBI = M[B][:, I]
    lu = spla.splu(MII)
    UI = lu.solve(-(MIB @ G))
    return (MBB @ G + MBI @ UI) / h


def solution_apply(n: int, R: np.ndarray, b=None, c=None, d=None, conv: str = "central",
                   M: sp.csr_matrix = None, ring_rows: str = "R2", form: str = "pde") -> np.ndarray:
    """X = S'^{-1} R (ring order): the ring part of the solution of M' x = r_hat, r_hat = R on the ring
    and 0 at the interior nodes.  With the R2 ring rows M' is the h^2-scaled five-point matrix of the
    whole grid, so this is the paper's G R; h X is T^{-1} R for T = S'/h."""
    if M is None:
        M = assemble(n, b, c, d, conv, ring_rows, form)
    B, _ = ring_and_interior(n)
    R = np.asarray(R, dtype=np.float64)
    vec = R.ndim == 1
    if vec:
        R = R[:, None]
    rhat = np.zeros((n * n, R.shape[1]))
    rhat[B] = R
    X = spla.splu(M.tocsc()).solve(rhat)[B]
    return X[:, 0] if vec else X
