"""Seeded synthetic inputs for the DtN build/apply workloads.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
no part of the method's arithmetic: it only draws coefficient fields b, c, d
sampled at the grid nodes and Dirichlet data G, from numpy's PCG64 generator.

Grid convention (the paper's Section 7): an n x n grid of nodes
(x_i, y_j) = (i h, j h), h = 1/(n-1), on the unit square; a nodal field is a
flat float64 array of length n*n with node (i, j) at index i + n*j.  The
boundary ring has nb = 4(n-1) nodes.

The paper's own experiments use formula-defined problems (Section 7.1) and no
public dataset; the configurations below stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "node_xy", "fourier_field", "cd_coeffs", "helmholtz_d", "boundary_data",
    "Problem", "CONFIGS", "config", "serving_operators", "serving_requests", "serving_builds",
    "PAPER_PROBLEMS", "paper_problem", "laplace_eigenvalue", "ring_xy", "error_vectors",
]


def node_xy(n: int):
    """Node coordinates as two (n, n) arrays indexed [j, i] (row = y)."""
    t = np.arange(n, dtype=np.float64) / (n - 1)
    x, y = np.meshgrid(t, t, indexing="xy")
    return x, y


def fourier_field(n: int, seed: int, modes: int = 8, kmax: int = 4) -> np.ndarray:
    """Sum of `modes` random Fourier modes, wavenumbers <= kmax, amplitude <= 1.

    f(x, y) = sum_m a_m cos(2 pi (p_m x + q_m y) + phi_m), with (p_m, q_m)
    uniform on {-kmax..kmax}^2 minus (0, 0), a_m ~ U[-1, 1], phi_m ~ U[0, 2 pi).
    Returned flat, node (i, j) at index i + n*j.
    """
    rng = np.random.default_rng(seed)
    pairs = [(p, q) for p in range(-kmax, kmax + 1) for q in range(-kmax, kmax + 1) if (p, q) != (0, 0)]
    idx = rng.integers(0, len(pairs), size=modes)
    amp = rng.uniform(-1.0, 1.0, size=modes)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    x, y = node_xy(n)
    f = np.zeros((n, n), dtype=np.float64)
    for m in range(modes):
        p, q = pairs[idx[m]]
        f += amp[m] * np.cos(2.0 * math.pi * (p * x + q * y) + phase[m])
    return np.ascontiguousarray(f.reshape(-1))


def cd_coeffs(n: int, seeds=(2001, 2002, 2003)):
    """Variable-coefficient convection-diffusion fields (b, c, d); d shifted to be >= 0."""
    b = fourier_field(n, seeds[0])
    c = fourier_field(n, seeds[1])
    d = fourier_field(n, seeds[2])
    d = d - d.min()
    return b, c, d


def helmholtz_d(n: int, kappa: float) -> np.ndarray:
    """Constant field d = -kappa^2 (Helmholtz, b = c = 0)."""
    return np.full(n * n, -kappa * kappa, dtype=np.float64)


def boundary_data(nb: int, k: int, seed: int) -> np.ndarray:
    """k Dirichlet vectors, entries i.i.d. U[-1, 1]; column-major nb x k (Fortran order)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.uniform(-1.0, 1.0, size=(nb, k)))


def ring_xy(n: int):
    """Coordinates of the nb = 4(n-1) ring nodes in ring order: counter-clockwise from (0, 0), index
    r = s (n-1) + t with side s = 0 south (t, 0), 1 east (n-1, t), 2 north (n-1-t, n-1), 3 west
    (0, n-1-t), in grid units divided by n - 1."""
    t = np.arange(n - 1)
    i = np.concatenate([t, np.full(n - 1, n - 1), n - 1 - t, np.zeros(n - 1, dtype=int)])
    j = np.concatenate([np.zeros(n - 1, dtype=int), t, np.full(n - 1, n - 1), n - 1 - t])
    return i / (n - 1), j / (n - 1)


def error_vectors(n: int, seed: int = 7001) -> np.ndarray:
    """The two right-hand sides of the e1 / e2 errors (Section 7.1), nb x 2, column-major: a unit
    vector of uniformly random direction (normalised Gaussian), and a smooth one, the restriction of
    cos(pi x) + sin(2 pi y) + x y to the ring, normalised."""
    x, y = ring_xy(n)
    r1 = np.random.default_rng(seed).standard_normal(x.size)
    r2 = np.cos(math.pi * x) + np.sin(2.0 * math.pi * y) + x * y
    R = np.stack([r1 / np.linalg.norm(r1), r2 / np.linalg.norm(r2)], axis=1)
    return np.asfortranarray(R)


@dataclass
class Problem:
    """One build problem: grid size, leaf box side, coefficient fields (None = 0)."""
    name: str
    n: int
    leaf: int
    b: Optional[np.ndarray] = None
    c: Optional[np.ndarray] = None
    d: Optional[np.ndarray] = None
    kind: str = "laplace"
    k: int = 0              # number of Dirichlet vectors to apply
    g_seed: int = 0
    tol: float = 0.0
    meta: dict = field(default_factory=dict)
    form: str = "pde"       # "pde" (five-point PDE coefficients) or "network" (b, c: link conductances)

    @property
    def nb(self) -> int:
        return 4 * (self.n - 1)

    def G(self, k: Optional[int] = None) -> np.ndarray:
        return boundary_data(self.nb, self.k if k is None else k, self.g_seed)


def _cfg1():
    return Problem("laplace_n32_leaf8", 32, 8, kind="laplace", k=16, g_seed=1001)


def _cfg2():
    b, c, d = cd_coeffs(256, (2001, 2002, 2003))
    return Problem("convdiff_n256_leaf16", 256, 16, b, c, d, kind="convdiff", k=256, g_seed=2004)


def _cfg3():
    kappa = 40.0 * math.pi  # 20 wavelengths across the unit square
    return Problem("helmholtz20w_n1024_leaf32", 1024, 32, None, None, helmholtz_d(1024, kappa),
                   kind="helmholtz", k=1024, g_seed=3001, meta={"kappa": kappa})


def _cfg4(instance: str = "convdiff"):
    if instance == "laplace":
        return Problem("laplace_n2048_leaf32", 2048, 32, kind="laplace", k=256, g_seed=4004, tol=1e-10)
    b, c, d = cd_coeffs(2048, (4001, 4002, 4003))
    return Problem("convdiff_n2048_leaf32", 2048, 32, b, c, d, kind="convdiff", k=256, g_seed=4004, tol=1e-10)


CONFIGS = {"cfg1": _cfg1, "cfg2": _cfg2, "cfg3": _cfg3, "cfg4": _cfg4}

# The eleven problems of the paper's Section 7.1, by name.
PAPER_PROBLEMS = ("laplace", "diffconv1", "diffconv2", "diffconv3", "diffconv4", "helmholtz1", "helmholtz2",
                  "helmholtz3", "helmholtz4", "randlap1", "randlap2")


def laplace_eigenvalue(n: int, index: int) -> float:
    """The index-th (from 1, ascending, with multiplicity) eigenvalue of the discrete Dirichlet Laplacian
    on the (n-2) x (n-2) interior nodes, h = 1/(n-1): (4/h^2)(sin^2(p pi h/2) + sin^2(q pi h/2))."""
    h = 1.0 / (n - 1)
    s = np.sin(np.arange(1, n - 1) * math.pi * h / 2.0) ** 2
    m = min(n - 2, index + 1)                  # the index smallest need p, q <= index
    lam = np.sort((s[:m, None] + s[None, :m]).ravel()) * 4.0 / (h * h)
    return float(lam[index - 1])


def paper_problem(name: str, n: int, leaf: int = 32, seed: int = 6001) -> Problem:
    """One of the Section 7.1 problems on an n x n grid (coefficients at the nodes; Random Laplacians
    as link conductances drawn from `seed`)."""
    x, y = node_xy(n)
    x, y = x.reshape(-1), y.reshape(-1)
    const = lambda v: np.full(n * n, float(v))
    if name == "laplace":
        return Problem(f"{name}_n{n}", n, leaf, kind=name)
    if name in ("diffconv1", "diffconv2"):
        return Problem(f"{name}_n{n}", n, leaf, const(100.0 if name == "diffconv1" else 1000.0), None, None, kind=name)
    if name == "diffconv3":      # divergence-free convection
        return Problem(f"{name}_n{n}", n, leaf, 125.0 * np.cos(4 * math.pi * y), 125.0 * np.sin(4 * math.pi * x), None,
                       kind=name)
    if name == "diffconv4":      # convection with sources and sinks
        return Problem(f"{name}_n{n}", n, leaf, 125.0 * np.cos(4 * math.pi * x), 125.0 * np.sin(4 * math.pi * y), None,
                       kind=name)
    if name == "helmholtz1":
        return Problem(f"{name}_n{n}", n, leaf, None, None, const(-100.0), kind=name)
    if name == "helmholtz2":
        return Problem(f"{name}_n{n}", n, leaf, None, None, const(-4005.0), kind=name)
    if name == "helmholtz3":     # next to the tenth eigenvalue of the discrete Laplacian
        lam = laplace_eigenvalue(n, 10)
        return Problem(f"{name}_n{n}", n, leaf, None, None, const(-lam + 1e-5), kind=name, meta={"lambda10": lam})
    if name == "helmholtz4":     # 40 points per wavelength
        return Problem(f"{name}_n{n}", n, leaf, None, None, const(-(2 * math.pi * n / 40.0) ** 2), kind=name)
    if name in ("randlap1", "randlap2"):
        rng = np.random.default_rng(seed)
        hi = 2.0 if name == "randlap1" else 1000.0
        return Problem(f"{name}_n{n}", n, leaf, rng.uniform(1.0, hi, n * n), rng.uniform(1.0, hi, n * n), None,
                       kind=name, form="network")
    raise ValueError(name)


def config(name: str, *args) -> Problem:
    return CONFIGS[name](*args)


def serving_operators(seed: int = 5001):
    """The eight resident operators of the serving workload.

    (n, leaf, kind): (128,16,L) (128,16,CD) (256,16,H) (256,16,CD) (512,32,L)
    (512,32,H) (1024,32,CD) (1024,32,L).  Helmholtz operators use
    kappa = 2 pi w with w = U[0.9, 1.0] * (n-1)/25 wavelengths.
    """
    rng = np.random.default_rng(seed)
    spec = [(128, 16, "laplace"), (128, 16, "convdiff"), (256, 16, "helmholtz"), (256, 16, "convdiff"),
            (512, 32, "laplace"), (512, 32, "helmholtz"), (1024, 32, "convdiff"), (1024, 32, "laplace")]
    ops = []
    for q, (n, leaf, kind) in enumerate(spec):
        if kind == "laplace":
            ops.append(Problem(f"op{q}_laplace_n{n}", n, leaf, kind=kind))
        elif kind == "convdiff":
            s = int(rng.integers(0, 10**6))
            b, c, d = cd_coeffs(n, (s, s + 1, s + 2))
            ops.append(Problem(f"op{q}_convdiff_n{n}", n, leaf, b, c, d, kind=kind))
        else:
            w = rng.uniform(0.9, 1.0) * (n - 1) / 25.0
            kappa = 2.0 * math.pi * w
            ops.append(Problem(f"op{q}_helmholtz_n{n}", n, leaf, None, None, helmholtz_d(n, kappa),
                               kind=kind, meta={"kappa": kappa}))
    return ops


def serving_builds(count: int, p: float = 0.002, seed: int = 5200):
    """Which arrivals of the serving stream are build requests (probability p each) and the problem of
    each: n ~ U{128, 256} (leaf 16), PDE ~ U{Laplace, convection-diffusion, Helmholtz} with seeded
    coefficients (Helmholtz: kappa = 2 pi w, w ~ U[0.9, 1.0] (n-1)/25).  Returns {arrival index: Problem}."""
    rng = np.random.default_rng(seed)
    picks = np.nonzero(rng.uniform(0.0, 1.0, count) < p)[0]
    out = {}
    for q in picks:
        n = int(rng.choice([128, 256]))
        kind = ("laplace", "convdiff", "helmholtz")[int(rng.integers(0, 3))]
        if kind == "laplace":
            out[int(q)] = Problem(f"build{q}_laplace_n{n}", n, 16, kind=kind)
        elif kind == "convdiff":
            s = int(rng.integers(0, 10**6))
            b, c, d = cd_coeffs(n, (s, s + 1, s + 2))
            out[int(q)] = Problem(f"build{q}_convdiff_n{n}", n, 16, b, c, d, kind=kind)
        else:
            kappa = 2.0 * math.pi * rng.uniform(0.9, 1.0) * (n - 1) / 25.0
            out[int(q)] = Problem(f"build{q}_helmholtz_n{n}", n, 16, None, None, helmholtz_d(n, kappa), kind=kind)
    return out


def serving_requests(count: int = 10000, nops: int = 8, seed: int = 5100, k_seed: int = 5101, kmax: int = 64):
    """Request stream of the serving workload: unit-rate Poisson inter-arrival gaps (scale by
    1/lambda), operator ~ U{0..nops-1}, k ~ U{1..kmax}.  Returns (gaps, op, k) arrays."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0, count)
    op = rng.integers(0, nops, count)
    k = np.random.default_rng(k_seed).integers(1, kmax + 1, count)
    return gaps, op, k
