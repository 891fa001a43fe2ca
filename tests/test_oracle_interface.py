"""CPU pins of the interface pair order used by the structured merges (Section 6, Step 1).

The merge's interface block K_ii = [[S33, A34], [A43, S44]] couples the two children's interface lines
through the stencil: A34 is anti-diagonal (the lines run along the shared edge in opposite directions),
so in the plain order its off-diagonal half is a full-rank block, while in the pair order (each P3 node
followed by its neighbour in P4) the off-diagonal blocks of the binary tree have low rank.  Solving the
merge through the oracle's Algorithms 1 and 2 in the pair order must reproduce the merge's Schur
complement at the scale of the tolerance.
"""
import numpy as np
import pytest

from interface_block import root_merge_blocks
from oracle.hbs import hbs_compress_square, hbs_invert, hbs_inverse_apply


def _rank(A, tol):
    s = np.linalg.svd(A, compute_uv=False)
    return int((s > tol * s[0]).sum()) if s.size and s[0] > 0 else 0


def _coeffs(kind, n):
    rng = np.random.default_rng(n)
    if kind == "cd":
        return rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    if kind == "helm":
        return None, None, np.full(n * n, -300.0)
    return None, None, None


@pytest.mark.parametrize("which", ["root", "bottom"])
def test_pair_order_structure(which):
    n = 129
    B = root_merge_blocks(n, *_coeffs("cd", n), leaf=16, which=which)
    Kii, i1, src = B["Kii"], B["i1"], B["pair"]
    i = Kii.shape[0]
    assert i == 2 * i1 and np.array_equal(np.sort(src), np.arange(i))
    A34 = Kii[:i1, i1:]
    # anti-diagonal coupling with nonzero entries: full rank in the plain order
    assert np.count_nonzero(A34 - np.fliplr(np.diag(np.diag(np.fliplr(A34))))) == 0
    assert np.all(np.diag(np.fliplr(A34)) != 0)
    assert _rank(A34, 1e-12) == i1
    # pair order: partners adjacent, low-rank off-diagonal blocks at every split of the tree
    K = Kii[np.ix_(src, src)]
    assert np.all(src[1::2] - i1 == i1 - 1 - src[0::2])          # the partner of P3[r] is P4[i1-1-r]
    h = i // 2
    assert _rank(K[:h, h:], 1e-10) <= 40 and _rank(K[h:, :h], 1e-10) <= 40
    q = i // 4
    assert _rank(np.hstack([K[:q, q:], K[q:, :q].T]), 1e-10) <= 60


@pytest.mark.parametrize("kind,tol,bound", [("laplace", 1e-10, 1e-9), ("cd", 1e-10, 1e-9), ("helm", 1e-12, 1e-9)])
def test_pair_order_algorithm1_reproduces_merge(kind, tol, bound):
    n = 129
    B = root_merge_blocks(n, *_coeffs(kind, n), leaf=16)
    Kii, Kie, Kei, Kee, src = B["Kii"], B["Kie"], B["Kei"], B["Kee"], B["pair"]
    S_ref = Kee - Kei @ np.linalg.solve(Kii, Kie)
    Xp = hbs_inverse_apply(hbs_invert(hbs_compress_square(Kii[np.ix_(src, src)], 32, tol)), Kie[src])
    X = np.empty_like(Xp)
    X[src] = Xp
    S = Kee - Kei @ X
    err = np.linalg.norm(S - S_ref) / np.linalg.norm(S_ref)
    assert err <= bound, err
    # a wrong scatter of the rows (X left in the pair order) is caught
    bad = np.linalg.norm(Kee - Kei @ Xp - S_ref) / np.linalg.norm(S_ref)
    assert bad > 1e-3


@pytest.mark.parametrize("kind", ["laplace", "cd", "helm"])
def test_structured_nd_build(kind):
    """The oracle's build with its top three merges structured (children's rings >= 200 at n = 129)
    against the closed form (Laplace) or the LU build, at the scale of the local tolerance."""
    from oracle import dst_dtn, nd_dtn
    n = 129
    b, c, d = _coeffs(kind, n)
    T = nd_dtn(n, b, c, d, leaf=16, kii_tol=1e-10 if kind != "helm" else 1e-12, kii_min_ring=200)
    ref = dst_dtn(n, 0.0) if kind == "laplace" else nd_dtn(n, b, c, d, leaf=16)
    err = np.linalg.norm(T - ref) / np.linalg.norm(ref)
    assert err <= 1e-9, err
    # the structured merges ran: the result differs from the LU build at rounding scale or above
    if kind != "laplace":
        assert err > 0.0
