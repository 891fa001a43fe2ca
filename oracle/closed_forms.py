"""Closed forms of the discrete DtN operator (oracle).

For b = c = 0 and constant d the five-point problem separates.  Take
Dirichlet data supported on one edge of the square, equal to the discrete sine
mode sin(p pi t h) at the edge node t (t = 1..n-2), and zero on the rest of
the ring.  With a the distance (in nodes) from that edge, the discrete
solution is u(a, t) = X_a sin(p pi t h) where

    X_{a+1} + X_{a-1} = 2 lam X_a,   lam = 2 + h^2 d / 2 - cos(p pi h),
    X_0 = 1,  X_{n-1} = 0,

so X_a is a ratio of sinh (lam > 1), of sin (|lam| < 1), alternating sinh
(lam < -1) or linear (|lam| = 1) functions.  The operator then follows from
its definition (T g)(b) = (g(b) - u(b_in)) / h on each edge, and the modes
p = 1..n-2 of the four edges span the ring minus its corners (the discrete
sine transform of type I is orthogonal), so T is known entry by entry.

X_a is evaluated in numpy.longdouble by default, so that near an interior
resonance the oracle's own rounding stays below the problem's conditioning;
the final sine-transform sum is done in float64.
"""
from __future__ import annotations

import numpy as np

from .grid import ring_nodes


def trace_on_ring(n: int, f) -> np.ndarray:
    """Values f(x, y) at the ring nodes (counter-clockwise from (0,0)); f vectorised."""
    h = 1.0 / (n - 1)
    pts = np.array(ring_nodes(n), dtype=np.float64)
    return np.asarray(f(pts[:, 0] * h, pts[:, 1] * h), dtype=np.float64)


def _profile(n: int, lam: np.ndarray, dtype) -> np.ndarray:
    """X[a, q] for a = 0..n-1 solving the three-term recurrence with X_0 = 1, X_{n-1} = 0."""
    lam = lam.astype(dtype)
    a = np.arange(n, dtype=dtype)[:, None]
    N1 = dtype(n - 1)
    X = np.zeros((n, lam.size), dtype=dtype)
    one = dtype(1)
    for sgn_region in ("gt", "lt", "in", "eq1", "eqm1"):
        if sgn_region == "gt":
            m = lam > one
            mu = lam[m]
        elif sgn_region == "lt":
            m = lam < -one
            mu = -lam[m]
        elif sgn_region == "in":
            m = (lam > -one) & (lam < one)
        elif sgn_region == "eq1":
            m = lam == one
        else:
            m = lam == -one
        if not np.any(m):
            continue
        if sgn_region in ("gt", "lt"):
            th = np.arccosh(mu)[None, :]
            # sinh(th (N1 - a)) / sinh(th N1), in overflow-free form
            num = -np.expm1(-2 * th * (N1 - a))
            den = -np.expm1(-2 * th * N1)
            Xm = np.exp(-th * a) * num / den
            if sgn_region == "lt":
                Xm = Xm * np.where((np.arange(n) % 2) == 0, one, -one).astype(dtype)[:, None]
        elif sgn_region == "in":
            ph = np.arccos(lam[m])[None, :]
            Xm = np.sin(ph * (N1 - a)) / np.sin(ph * N1)
        else:
            Xm = np.repeat((N1 - a) / N1, int(m.sum()), axis=1)
            if sgn_region == "eqm1":
                Xm = Xm * np.where((np.arange(n) % 2) == 0, one, -one).astype(dtype)[:, None]
        X[:, m] = Xm
    return X


def dst_dtn(n: int, d: float = 0.0, dtype=np.longdouble) -> np.ndarray:
    """Full T (nb x nb, ring order counter-clockwise from (0,0)) for b = c = 0, constant d."""
    if n < 3:
        raise ValueError("n must be >= 3")
    h = 1.0 / (n - 1)
    nb = 4 * (n - 1)
    ring = ring_nodes(n)
    p = np.arange(1, n - 1)
    hd = dtype(h)
    pi = dtype(np.pi) if dtype is np.float64 else np.arccos(dtype(-1))
    lam = dtype(2) + hd * hd * dtype(d) / 2 - np.cos(p.astype(dtype) * pi * hd)
    X = _profile(n, lam, dtype)                                  # (n, n-2)
    t = np.arange(1, n - 1)
    sin_pt = np.sin(np.outer(t.astype(dtype), p.astype(dtype)) * pi * hd)   # [t-1, p-1]
    sin_p1 = np.sin(p.astype(dtype) * pi * hd)
    sin_pn = np.sin(p.astype(dtype) * pi * hd * dtype(n - 2))
    a = np.arange(1, n - 1)

    # edge maps (a, t) -> (i, j) for the W, E, S, N edges
    maps = [
        lambda A, T_: (A, T_),
        lambda A, T_: (n - 1 - A, T_),
        lambda A, T_: (T_, A),
        lambda A, T_: (T_, n - 1 - A),
    ]

    rarr = np.full((n, n), -1, dtype=np.int64)                   # rarr[i, j] = ring index
    for r, (i_, j_) in enumerate(ring):
        rarr[i_, j_] = r

    def ridx_of(i, j):
        i, j = np.broadcast_arrays(np.asarray(i), np.asarray(j))
        return rarr[i, j]

    T = np.zeros((nb, nb))
    for f in maps:
        Y = np.zeros((nb, n - 2), dtype=dtype)
        # the edge itself (a = 0): (g - u(1, t)) / h
        i0, j0 = f(0, t)
        r_edge = ridx_of(i0, j0)
        Y[r_edge, :] = sin_pt * (1 - X[1, :])[None, :] / hd
        # the opposite edge (a = n-1): -u(n-2, t) / h
        i1, j1 = f(n - 1, t)
        Y[ridx_of(i1, j1), :] = -sin_pt * X[n - 2, :][None, :] / hd
        # the two adjacent edges (t = 0 and t = n-1), nodes a = 1..n-2
        i2, j2 = f(a, 0)
        Y[ridx_of(i2, j2), :] = -X[1:n - 1, :] * sin_p1[None, :] / hd
        i3, j3 = f(a, n - 1)
        Y[ridx_of(i3, j3), :] = -X[1:n - 1, :] * sin_pn[None, :] / hd
        # unit vector at edge node t0 = sum_p (2/(n-1)) sin(p pi t0 h) * mode p
        coef = (2.0 / (n - 1)) * sin_pt.astype(np.float64).T          # [p-1, t0-1]
        T[:, r_edge] = Y.astype(np.float64) @ coef
    return T
