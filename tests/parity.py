"""Element-wise comparison of a GPU result with its reference.

A relative Frobenius error alone can hide an error concentrated in one row or
one entry (a corner, an interface node, a mis-gathered arc), so every GPU
comparison also bounds
  entry: max |A - R| / max |R|                  (the worst entry, relative to the largest one)
  row:   max_r ||(A - R)[r, :]|| / max_r ||R[r, :]||   (the worst row)
The entry bound defaults to the Frobenius tolerance.  The row bound defaults to
twice it: the rows of a DtN operator have similar norms, so an error spread
over the rows gives row ~ fro, while an error held in one row of an nb-row
operator gives row ~ sqrt(nb) fro; a factor of two admits only mild
concentration (the error of a near-resonant problem gathers on the rows where
its smooth resonant modes live).
"""
from __future__ import annotations

import numpy as np


def errors(A, R) -> dict:
    A = np.asarray(A, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    assert A.shape == R.shape, (A.shape, R.shape)
    D = A - R
    nR = np.linalg.norm(R)
    out = {"fro": float(np.linalg.norm(D) / max(nR, 1e-300))}
    out["entry"] = float(np.abs(D).max() / max(np.abs(R).max(), 1e-300)) if D.size else 0.0
    if D.ndim == 2 and D.size:
        out["row"] = float(np.linalg.norm(D, axis=1).max() / max(np.linalg.norm(R, axis=1).max(), 1e-300))
    else:
        out["row"] = out["entry"]
    return out


def assert_close(A, R, tol: float, entry: float | None = None, row: float | None = None, label: str = "") -> dict:
    e = errors(A, R)
    print(f"{label} fro {e['fro']:.3e} entry {e['entry']:.3e} row {e['row']:.3e}", flush=True)
    assert e["fro"] <= tol, (label, "fro", e)
    assert e["entry"] <= (tol if entry is None else entry), (label, "entry", e)
    assert e["row"] <= (2.0 * tol if row is None else row), (label, "row", e)
    return e
