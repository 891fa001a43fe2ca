"""GPU parity of the ring-row readings (DTN_RING_R1 / R2 / R3) through the C ABI.

The build eliminates the same interior for every reading; R2 and R3 change only the ring rows, which
the root output kernel applies to the root Schur complement.  Checked against the oracle's own
assembly of each reading (nested dissection on the matrix with those ring rows), across problems of
one fused multi-problem build, and at n = 1024 against the closed form plus the exact ring-row change.
"""
import math

import numpy as np
import pytest

from oracle import nd_dtn, dst_dtn, ring_nodes
from parity import assert_close

pytestmark = pytest.mark.gpu

READING = {"R1": 0, "R2": 1, "R3": 2}


def coeffs(n, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "laplace":
        return None, None, None
    if kind == "cd":
        return rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    return None, None, np.full(n * n, -rng.uniform(10, 300))


@pytest.mark.parametrize("rows", ["R2", "R3"])
@pytest.mark.parametrize("n,leaf,kind", [(17, 8, "cd"), (64, 16, "laplace"), (130, 32, "cd"), (97, 16, "helm")])
def test_ring_rows_vs_oracle(dtn, n, leaf, kind, rows):
    b, c, d = coeffs(n, kind, 40 + n)
    op = dtn.build(n, b, c, d, leaf=leaf, ring_rows=READING[rows])
    T = op.dense()
    op.free()
    assert_close(T, nd_dtn(n, b, c, d, leaf=leaf, ring_rows=rows), 1e-10, label=f"{rows} n={n} {kind}")


def test_ring_rows_paper_convection_scale(dtn):
    n = 41
    b, c, d = coeffs(n, "cd", 9)
    op = dtn.build(n, b, c, d, leaf=8, conv=dtn.CONV_PAPER, ring_rows=dtn.RING_R2)
    assert_close(op.dense(), nd_dtn(n, b, c, d, leaf=8, conv="paper", ring_rows="R2"), 1e-10, label="R2 paper conv")
    op.free()


def test_ring_rows_mixed_in_one_fused_build(dtn):
    probs = [(33, 8, "cd", "R2"), (64, 16, "laplace", "R3"), (45, 8, "cd", "R1"), (50, 16, "helm", "R2")]
    specs, refs = [], []
    for q, (n, leaf, kind, rows) in enumerate(probs):
        b, c, d = coeffs(n, kind, 70 + q)
        specs.append(dict(n=n, b=b, c=c, d=d, leaf=leaf, ring_rows=READING[rows]))
        refs.append(nd_dtn(n, b, c, d, leaf=leaf, ring_rows=rows))
    ops = dtn.build_many(specs)
    for (n, leaf, kind, rows), op, Tref in zip(probs, ops, refs):
        assert_close(op.dense(), Tref, 1e-10, label=f"many {rows} n={n}")
        op.free()


@pytest.mark.parametrize("d", [0.0, -(40.0 * math.pi) ** 2])
def test_ring_rows_full_size_closed_form(dtn, d):
    """n = 1024, leaf 32: R3 = closed-form T + (cycle Laplacian)/h; R2 = closed-form T + (the ring-ring
    block of the five-point rows)/h, both exact identities for b = c = 0."""
    n = 1024
    h = 1.0 / (n - 1)
    dd = None if d == 0.0 else np.full(n * n, d)
    T1 = dst_dtn(n, d)
    nb = 4 * (n - 1)
    ring = ring_nodes(n)
    corner = np.array([i in (0, n - 1) and j in (0, n - 1) for (i, j) in ring])
    nxt = (np.arange(nb) + 1) % nb
    prv = (np.arange(nb) - 1) % nb
    for rows in ("R3", "R2"):
        op = dtn.build(n, None, None, dd, leaf=32, ring_rows=READING[rows])
        T = op.dense()
        op.free()
        ref = T1.copy()
        diag = 2.0 if rows == "R3" else np.where(corner, 4.0, 3.0) + h * h * d
        ref[np.arange(nb), np.arange(nb)] += diag / h
        ref[np.arange(nb), nxt] += -1.0 / h
        ref[np.arange(nb), prv] += -1.0 / h
        assert_close(T, ref, 1e-10, label=f"{rows} n=1024 d={d}")
