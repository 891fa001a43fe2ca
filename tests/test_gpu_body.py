"""GPU tests of the body-load operator F of Section 7.3 (v = T g + F f_hat): the loads' condensed
right-hand sides carried through the leaf elimination and every merge (Section 3.2's update), against the
oracle's definition F = h M'_BI M'_II^{-1} P (one sparse solve), on the fast and the partially pivoted
paths, for the PDE and network forms; T itself is unchanged by the loads."""
import numpy as np
import pytest

import workloads as W
from oracle.body import body_operator
from parity import assert_close

pytestmark = pytest.mark.gpu


def _loads(n, count, seed, leaf, box=None):
    rng = np.random.default_rng(seed)
    lo, hi = (1, n - 1) if box is None else box
    pts = set()
    while len(pts) < count:
        pts.add((int(rng.integers(lo, hi)), int(rng.integers(lo, hi))))
    # loads on box rings, at a box corner and next to the grid's ring
    for p in ((leaf - 1, leaf - 1), (leaf, 3), (1, n // 2), (n - 2, n - 2), (n // 2, n // 2)):
        if box is None:
            pts.add(p)
    return sorted(pts)


@pytest.mark.parametrize("n,leaf,kind,pivoting", [
    (65, 8, "cd", "auto"), (129, 16, "helm", "auto"), (129, 16, "cd", "partial"), (257, 32, "laplace", "auto")])
def test_body_operator_vs_oracle(dtn, n, leaf, kind, pivoting):
    rng = np.random.default_rng(n + 1)
    b = c = d = None
    if kind == "cd":
        b, c, d = rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    elif kind == "helm":
        d = np.full(n * n, -(2 * np.pi * 4) ** 2)
    nodes = _loads(n, 24, n, leaf)
    piv = dtn.PIVOT_PARTIAL if pivoting == "partial" else dtn.PIVOT_AUTO
    op = dtn.build(n, b, c, d, leaf=leaf, pivoting=piv, body_nodes=nodes)
    assert op.body_count == len(nodes)
    F = op.body()
    T = op.dense()
    op.free()
    Fr = body_operator(n, nodes, b, c, d)
    assert_close(F, Fr, 1e-10, label=f"F n={n} {kind} {pivoting}")
    plain = dtn.build(n, b, c, d, leaf=leaf, pivoting=piv)
    assert np.array_equal(T, plain.dense())
    plain.free()


def test_body_operator_network_form_localized(dtn):
    """The random Laplacian of Section 7.3's experiment (network form, conductances U[1, 2]) with 100
    loads in a localized square; with d = 0 every unit load's fluxes add up to -h."""
    n = 257
    P = W.paper_problem("randlap1", n)
    nodes = _loads(n, 100, 7, 32, box=(96, 160))
    op = dtn.build(n, P.b, P.c, P.d, leaf=32, coef_form=dtn.COEF_NETWORK, body_nodes=nodes)
    F = op.body()
    op.free()
    Fr = body_operator(n, nodes, P.b, P.c, P.d, form="network")
    assert_close(F, Fr, 1e-10, label="F randlap1 n=257")
    assert np.allclose(F.sum(axis=0), -1.0 / (n - 1), rtol=0, atol=1e-12)


def test_body_apply_and_columns_in_caller_order(dtn):
    import torch
    n = 129
    nodes = [(100, 20), (5, 5), (64, 64), (30, 90)]          # not in quadtree order
    op = dtn.build(n, leaf=16, body_nodes=nodes)
    F = op.body()
    for q, p in enumerate(nodes):
        assert_close(F[:, q:q + 1], body_operator(n, [p]), 1e-10, label=f"column {q}")
    T = op.dense()
    rng = np.random.default_rng(3)
    G, Q = rng.uniform(-1, 1, (op.nb, 5)), rng.uniform(-1, 1, (len(nodes), 5))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()
    Y = op.apply_body_device(dev(G), dev(Q)).cpu().numpy()
    assert_close(Y, T @ G + F @ Q, 1e-12, label="T G + F Q")
    op.free()


def test_body_option_checks(dtn):
    with pytest.raises(dtn.DtnError):
        dtn.build(33, leaf=8, tol=1e-8, body_nodes=[(5, 5)])          # dense builds only
    with pytest.raises(dtn.DtnError):
        dtn.build(33, leaf=8, body_nodes=[(0, 5)])                   # a ring node
    with pytest.raises(dtn.DtnError):
        dtn.build(33, leaf=8, ring_rows=dtn.RING_R2, body_nodes=[(5, 5)])
    with pytest.raises(dtn.DtnError):
        dtn.build_many([dict(n=33, leaf=8, body_nodes=[(5, 5)]), dict(n=33, leaf=8)])
    op = dtn.build(33, leaf=8)
    assert op.body_count == 0
    with pytest.raises(dtn.DtnError):
        op.body()
    op.free()
