"""CPU pins of the body-load operator F of Section 7.3 (v = T g + F f_hat): its definition against a dense
inverse, an exact discrete conservation law, and the nested dissection that carries the loads' right-hand
sides through every merge (Section 3.2's update) against the definition."""
import numpy as np
import pytest

from oracle import assemble, nd_dtn
from oracle.assemble import ring_and_interior
from oracle.body import body_nested, body_operator


def _nodes(n, count, seed):
    rng = np.random.default_rng(seed)
    pts = set()
    while len(pts) < count:
        pts.add((int(rng.integers(1, n - 1)), int(rng.integers(1, n - 1))))
    return sorted(pts)


def test_definition_against_dense_inverse():
    n = 9
    rng = np.random.default_rng(1)
    b, c, d = rng.uniform(-3, 3, n * n), rng.uniform(-3, 3, n * n), rng.uniform(0, 5, n * n)
    nodes = [(1, 1), (4, 4), (7, 2), (3, 6)]
    F = body_operator(n, nodes, b, c, d)
    M = assemble(n, b, c, d).toarray()
    B, I = ring_and_interior(n)
    h = 1.0 / (n - 1)
    P = np.zeros((len(I), len(nodes)))
    for q, (i, j) in enumerate(nodes):
        P[list(I).index(i + n * j), q] = 1.0
    ref = h * M[np.ix_(B, I)] @ np.linalg.inv(M[np.ix_(I, I)]) @ P
    assert np.abs(F - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("form", ["pde", "network"])
def test_flux_of_a_unit_load_sums_to_minus_h(form):
    """With d = 0 and a symmetric operator every unit load's boundary fluxes add up to -h exactly: the
    interior rows of M' sum (over the rows) to the links toward the ring, so sum_b v_b = -h sum f_hat."""
    n = 17
    rng = np.random.default_rng(2)
    b = c = None
    if form == "network":
        b, c = rng.uniform(1, 2, n * n), rng.uniform(1, 2, n * n)
    nodes = _nodes(n, 6, 3)
    F = body_operator(n, nodes, b, c, None, form=form)
    h = 1.0 / (n - 1)
    assert np.allclose(F.sum(axis=0), -h, rtol=0, atol=1e-13)
    # and the fluxes point into the domain's sink (all <= 0) for the positive load
    assert np.all(F <= 1e-15)


@pytest.mark.parametrize("n,leaf,kind", [(33, 8, "laplace"), (33, 8, "cd"), (40, 8, "helm"), (65, 16, "cd")])
def test_nested_dissection_carries_the_loads(n, leaf, kind):
    rng = np.random.default_rng(n)
    b = c = d = None
    if kind == "cd":
        b, c, d = rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    elif kind == "helm":
        d = np.full(n * n, -200.0)
    # random nodes plus nodes on leaf rings, at a leaf corner and next to the grid's ring
    nodes = sorted(set(_nodes(n, 12, 4) + [(leaf - 1, leaf - 1), (leaf, 3), (1, n // 2), (n - 2, n - 2)]))
    T, F = body_nested(n, nodes, b, c, d, leaf=leaf)
    Fr = body_operator(n, nodes, b, c, d)
    assert np.abs(F - Fr).max() <= 1e-11 * np.abs(Fr).max()
    Tr = nd_dtn(n, b, c, d, leaf=leaf)
    assert np.abs(T - Tr).max() <= 1e-11 * np.abs(Tr).max()
