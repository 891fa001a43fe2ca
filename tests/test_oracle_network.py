"""Oracle pins for the network form (Section 7.1's random Laplacians) and the Section 7.1 problem
generators.

* Unit conductances give exactly the Laplace matrix.
* A random network's operator: three eliminations agree (dense Schur complement, sparse LU, nested
  dissection); it is symmetric (each link's conductance enters both of its rows); constants are in its
  null space (every interior row sums to zero, and so does every row of S').
* The discrete Laplacian's eigenvalues of the Helmholtz III problem: the first is (8/h^2) sin^2(pi h/2),
  the tenth (the (1,4) pair) (4/h^2)(sin^2(pi h/2) + sin^2(2 pi h)).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import assemble, brute_dtn, nd_dtn, sparse_apply


def test_unit_conductances_are_laplace():
    n = 17
    one = np.ones(n * n)
    A = assemble(n, one, one, None, form="network").toarray()
    L = assemble(n).toarray()
    assert np.array_equal(A, L)


@pytest.mark.parametrize("name,n,leaf", [("randlap1", 17, 8), ("randlap2", 24, 6), ("randlap2", 33, 8)])
def test_network_three_eliminations_agree(name, n, leaf):
    P = W.paper_problem(name, n, leaf=leaf)
    Tb = brute_dtn(n, P.b, P.c, P.d, form="network")
    Tn = nd_dtn(n, P.b, P.c, P.d, leaf=leaf, form="network")
    G = np.random.default_rng(n).uniform(-1, 1, (4 * (n - 1), 3))
    Ys = sparse_apply(n, G, P.b, P.c, P.d, form="network")
    scale = np.abs(Tb).max()
    assert np.abs(Tb - Tn).max() <= 1e-12 * scale
    assert np.abs(Ys - Tb @ G).max() <= 1e-12 * np.abs(Ys).max()
    assert np.abs(Tb - Tb.T).max() <= 1e-12 * scale
    assert np.abs(Tb.sum(axis=1)).max() <= 1e-11 * scale
    M = assemble(n, P.b, P.c, P.d, form="network").tocsr()
    inner = [i + n * j for j in range(1, n - 1) for i in range(1, n - 1)]
    assert np.abs(np.asarray(M[inner].sum(axis=1))).max() <= 1e-12 * P.b.max()


def test_network_rejects_r2():
    P = W.paper_problem("randlap1", 9, leaf=4)
    with pytest.raises(ValueError):
        assemble(9, P.b, P.c, None, ring_rows="R2", form="network")


@pytest.mark.parametrize("n", [33, 129, 1024])
def test_laplace_eigenvalues(n):
    h = 1.0 / (n - 1)
    assert W.laplace_eigenvalue(n, 1) == pytest.approx(8.0 / h ** 2 * math.sin(math.pi * h / 2) ** 2, rel=1e-13)
    want = 4.0 / h ** 2 * (math.sin(math.pi * h / 2) ** 2 + math.sin(2 * math.pi * h) ** 2)
    assert W.laplace_eigenvalue(n, 10) == pytest.approx(want, rel=1e-13)


def test_paper_problem_fields():
    n = 65
    x = np.arange(n) / (n - 1)
    P3 = W.paper_problem("diffconv3", n)
    assert P3.b.reshape(n, n)[:, 0] == pytest.approx(125 * np.cos(4 * math.pi * x))   # b = 125 cos(4 pi y)
    assert P3.c.reshape(n, n)[0, :] == pytest.approx(125 * np.sin(4 * math.pi * x))   # c = 125 sin(4 pi x)
    P4 = W.paper_problem("helmholtz4", n)
    assert P4.d[0] == pytest.approx(-(2 * math.pi * n / 40) ** 2)
    R = W.paper_problem("randlap2", n)
    assert R.form == "network" and 1.0 <= R.b.min() and R.b.max() <= 1000.0
    assert len(W.PAPER_PROBLEMS) == 11
