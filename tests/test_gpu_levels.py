"""GPU checks of intermediate quadtree levels and of the build budget, through the C ABI.

capture_level keeps the Schur complements of every box of one level as the build forms them
(Section 3.3).  Each box's S must equal the Schur complement of the assembled matrix restricted to the
box's nodes onto the box's ring (Section 3.1), computed here by a dense elimination of the oracle's
assembled matrix; this checks the leaves' in-box dissection, the merges of every level and the index
maps of the level buffers, element by element, with invariants that hold at every level: symmetry
without convection, and for Laplace boxes away from the grid's ring S 1 = the number of each ring node's
neighbours outside the box (the box's interior rows sum to zero).
The build budget: a build over budget fails with DTN_ENOMEM before allocating, one within it runs.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assemble, schur_complement
from oracle.grid import box_ring
from parity import assert_close

pytestmark = pytest.mark.gpu


def _box_schur(M, n, rect):
    x0, x1, y0, y1 = rect
    ring = [i + n * j for i, j in box_ring(x0, x1, y0, y1)]
    rs = set(ring)
    inner = [i + n * j for j in range(y0, y1) for i in range(x0, x1) if i + n * j not in rs]
    P = ring + inner
    A = M[P][:, P].toarray()
    m = len(ring)
    return schur_complement(A, np.arange(m), np.arange(m, len(P)))


@pytest.mark.parametrize("n,leaf,kind", [(65, 16, "laplace"), (65, 16, "cd"), (97, 32, "helm")])
def test_captured_levels_vs_dense_box_schur(dtn, n, leaf, kind):
    rng = np.random.default_rng(n)
    if kind == "cd":
        b, c, d = rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    elif kind == "helm":
        b, c, d = None, None, np.full(n * n, -300.0)
    else:
        b = c = d = None
    M = assemble(n, b, c, d)
    level = 0
    while True:
        try:
            op = dtn.build(n, b, c, d, leaf=leaf, capture_level=level)
        except dtn.DtnError as e:
            assert e.code == dtn.DTN_EINVAL and level >= 2      # deeper than the dissection
            break
        boxes = op.level_boxes()
        assert len(boxes) == 4 ** level
        worst = 0.0
        for rect, S in boxes:
            if level == 0:
                break                     # the whole grid: checked against T below
            R = _box_schur(M, n, rect)
            assert_close(S, R, 1e-11, label=f"n={n} {kind} level {level} box {rect}")
            worst = max(worst, np.abs(S - R).max() / np.abs(R).max())
            if b is None and c is None:
                assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
            x0, x1, y0, y1 = rect
            if kind == "laplace" and x0 > 0 and y0 > 0 and x1 < n and y1 < n:
                # a box away from the grid's ring: its interior rows sum to zero, so S 1 is the ring
                # rows' sums, the number of each ring node's neighbours outside the box (2 at corners)
                out = np.array([(i == x0) + (i == x1 - 1) + (j == y0) + (j == y1 - 1)
                                for i, j in box_ring(x0, x1, y0, y1)], dtype=float)
                assert np.abs(S.sum(axis=1) - out).max() <= 1e-11 * np.abs(S).max()
        print(f"n={n} {kind} level {level}: {len(boxes)} boxes, worst entry error {worst:.2e}", flush=True)
        if level == 0:
            # the root box's S is S' itself: T = S' / h
            assert_close(boxes[0][1] * (n - 1), op.dense(), 1e-14, label="root level vs T")
        op.free()
        level += 1
    assert level >= 3


def test_capture_in_fused_build(dtn):
    P1 = W.paper_problem("diffconv3", 65, leaf=16)
    ops = dtn.build_many([dict(n=65, b=P1.b, c=P1.c, leaf=16, capture_level=2),
                          dict(n=33, leaf=8, capture_level=1)])
    M1 = assemble(65, P1.b, P1.c, None)
    M2 = assemble(33)
    for rect, S in ops[0].level_boxes():
        assert_close(S, _box_schur(M1, 65, rect), 1e-11, label=f"fused, problem 0 box {rect}")
    for rect, S in ops[1].level_boxes():
        assert_close(S, _box_schur(M2, 33, rect), 1e-11, label=f"fused, problem 1 box {rect}")
    for op in ops:
        op.free()


def test_build_budget(dtn):
    n = 129
    with pytest.raises(dtn.DtnError) as e:
        dtn.build(n, leaf=16, budget_bytes=1)
    assert e.value.code == dtn.DTN_ENOMEM
    need = dtn.plan_footprint(n, leaf=16)[0] + (4 * (n - 1)) ** 2 * 8
    op = dtn.build(n, leaf=16, budget_bytes=max(need, 1))   # within the budget (plans possibly cached)
    T1 = op.dense()
    op.free()
    T2 = dtn.build(n, leaf=16).dense()
    assert np.array_equal(T1, T2)
    with pytest.raises(dtn.DtnError) as e:
        dtn.build(n, leaf=16, capture_level=1, budget_bytes=(4 * (n - 1)) ** 2 * 8)   # T fits, the level does not
    assert e.value.code == dtn.DTN_ENOMEM
