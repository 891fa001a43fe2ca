"""Pins for the oracle's HBS representation (Section 4: tree, def1-def6, telescoping tele1-tele3).

* Semiseparable matrices H = tril(u v^T) + triu(p q^T) + diag with rank-r generators are exactly HBS:
  every off-diagonal block row of a node is [lower part | upper part] of rank r per side, so the
  interpolative bases have exactly r columns per side of the node with a complement (2r inside,
  r at either end of the index range) wherever the node holds more rows than that, and the
  telescoping factorisation reproduces H to rounding.  A dropped sibling block, a transposed basis,
  a wrong skeleton index or a missed downward pass each break the reconstruction.
* The apply (upward pass, sibling blocks, downward pass, leaf blocks) equals H X for several X.
* On the closed-form DtN operator the reconstruction error sits at the tolerance's scale and the
  representation is several times smaller than the dense matrix (Table 2's memory, Section 7).
* The tree splits intervals of more than m indices into floor/ceil halves, children left then right.
"""
import numpy as np
import pytest

from oracle import dst_dtn
from oracle.hbs import hbs_tree, hbs_compress, hbs_apply, hbs_dense, hbs_words, hbs_ranks


def semiseparable(M, r, seed):
    rng = np.random.default_rng(seed)
    u, v, p, q = (rng.standard_normal((M, r)) for _ in range(4))
    return np.tril(u @ v.T, -1) + np.triu(p @ q.T, 1) + np.diag(rng.standard_normal(M))


def test_tree_halves():
    nodes = hbs_tree(300, 40)
    assert (nodes[0]["lo"], nodes[0]["hi"]) == (0, 300)
    leaves = [nd for nd in nodes if not nd["children"]]
    # every parent is split at lo + floor(len / 2), children left then right, leaves hold <= m
    for nd in nodes:
        if nd["children"]:
            a, b = (nodes[c] for c in nd["children"])
            mid = nd["lo"] + (nd["hi"] - nd["lo"]) // 2
            assert (a["lo"], a["hi"], b["lo"], b["hi"]) == (nd["lo"], mid, mid, nd["hi"])
            assert nd["hi"] - nd["lo"] > 40
        else:
            assert nd["hi"] - nd["lo"] <= 40
    assert sorted((nd["lo"], nd["hi"]) for nd in leaves) == [(nd["lo"], nd["hi"]) for nd in leaves]
    assert sum(nd["hi"] - nd["lo"] for nd in leaves) == 300


@pytest.mark.parametrize("M,m,r,seed", [(300, 20, 1, 1), (300, 20, 2, 2), (512, 32, 3, 3), (97, 10, 2, 4)])
def test_semiseparable_ranks_and_reconstruction(M, m, r, seed):
    H = semiseparable(M, r, seed)
    F = hbs_compress(H, m, 1e-12)
    for nd in F["nodes"][1:]:
        rows = (nd["hi"] - nd["lo"]) if not nd["children"] else sum(F["nodes"][c]["U"].shape[1] for c in nd["children"])
        sides = int(nd["lo"] > 0) + int(nd["hi"] < M)      # complement to the left, to the right
        assert nd["U"].shape[1] == min(sides * r, rows), (nd["lo"], nd["hi"], nd["U"].shape)
        assert nd["V"].shape[1] == min(sides * r, rows)
    assert np.abs(hbs_dense(F) - H).max() <= 1e-11 * np.abs(H).max()
    X = np.random.default_rng(seed + 9).standard_normal((M, 5))
    assert np.abs(hbs_apply(F, X) - H @ X).max() <= 1e-11 * np.abs(H @ X).max()
    assert np.allclose(hbs_apply(F, X[:, 0]), H @ X[:, 0], rtol=0, atol=1e-11 * np.abs(H @ X).max())


@pytest.mark.parametrize("tol", [1e-7, 1e-10])
def test_dtn_operator_at_tolerance(tol):
    n = 257
    T = dst_dtn(n, 0.0)
    F = hbs_compress(T, 64, tol)
    err = np.linalg.norm(hbs_dense(F) - T) / np.linalg.norm(T)
    assert err <= 10 * tol, err
    assert hbs_words(F) < T.size / 4
    ranks = hbs_ranks(F)
    assert ranks[0] == 0 and 0 < max(ranks) <= 64


# Algorithm 1 (inversion) and Algorithm 2 (application of the inverse), Section 5.1.
from oracle.hbs import hbs_compress_square, hbs_invert, hbs_inverse_apply  # noqa: E402
from oracle import brute_dtn  # noqa: E402


@pytest.mark.parametrize("M,m,r,seed", [(300, 20, 2, 5), (257, 16, 3, 6)])
def test_inverse_of_semiseparable_matrix(M, m, r, seed):
    """Exactly HBS (semiseparable generators plus a diagonal shift of 30, which keeps every node's
    compressed block V^* D~^{-1} U well conditioned, as Algorithm 1 assumes; with a shift of 10 some reach
    condition numbers ~1e6): Algorithm 2 on Algorithm 1's factors equals a dense solve to rounding;
    every node's row and column ranks are equal (Algorithm 1 inverts V^* D~^{-1} U)."""
    H = semiseparable(M, r, seed) + 30.0 * np.eye(M)
    F = hbs_compress_square(H, m, 1e-13)
    for nd in F["nodes"][1:]:
        assert nd["U"].shape[1] == nd["V"].shape[1]
    Fi = hbs_invert(F)
    X = np.random.default_rng(seed).standard_normal((M, 4))
    ref = np.linalg.solve(H, X)
    assert np.abs(hbs_inverse_apply(Fi, X) - ref).max() <= 1e-11 * np.abs(ref).max()


def test_inverse_of_r2_operator():
    """The paper's solution operator G = S^{-1} of the R2 ring rows (Section 3.1), at n = 33: from the
    HBS factors at tol 1e-10 against a dense solve, at the tolerance's scale times the conditioning."""
    n = 33
    T2 = brute_dtn(n, ring_rows="R2")
    F = hbs_compress_square(T2, 16, 1e-10)
    Fi = hbs_invert(F)
    X = np.random.default_rng(3).standard_normal((T2.shape[0], 3))
    ref = np.linalg.solve(T2, X)
    err = np.linalg.norm(hbs_inverse_apply(Fi, X) - ref) / np.linalg.norm(ref)
    assert err <= 1e-8, err


def test_inverse_of_convection_operator():
    """A divergence-free convection problem of Section 7.1 (diffusion-convection III) at n = 64, R2 rows:
    T is well conditioned, and the inverse from the joint-skeleton factors at tol 1e-10 must match a dense
    solve at the tolerance's scale (separate row and column skeletons made equal by forcing lose the
    result here: V^* D~^{-1} U becomes nearly singular)."""
    import workloads as W
    n = 64
    P = W.paper_problem("diffconv3", n, leaf=16)
    T = brute_dtn(n, P.b, P.c, P.d, ring_rows="R2")
    assert np.linalg.cond(T) < 100
    F = hbs_compress_square(T, 32, 1e-10)
    for nd in F["nodes"][1:]:
        assert np.array_equal(nd["J"], nd["Jc"]) and np.array_equal(nd["U"], nd["V"])
    X = np.random.default_rng(4).standard_normal((T.shape[0], 3))
    ref = np.linalg.solve(T, X)
    err = np.linalg.norm(hbs_inverse_apply(hbs_invert(F), X) - ref) / np.linalg.norm(ref)
    assert err <= 1e-8, err
