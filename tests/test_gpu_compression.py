"""GPU tests of the low-rank compressed merges (Section 6, Step 2) through the C ABI.

The off-diagonal child blocks S13, S31, S24, S42 of the top merges are replaced by factors
Q B found by a randomized range finder truncated at the build tolerance; the Schur update uses
the factored products.  Checked: the operator against the oracle / closed form at the
tolerance's scale, the ranks against the oracle's column-pivoted-QR ranks of the same blocks
(a different rank-revealing method: equal up to a few), the default level rule (children's
S >= 1000), the n = 2048 configuration against the oracle (Laplace: the closed form;
convection-diffusion: four columns of the operator from the oracle's sparse direct solve, stored by
tests/golden/make_cfg4_columns.py), and the rank cap reported as an error.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import nd_dtn, dst_dtn, assemble
from oracle.grid import build_tree, box_ring
from oracle.nd import box_schur, _interior_to_union
from oracle.hbs import pivoted_qr_rank
from parity import assert_close

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n,leaf,kind,tol,level,bound", [
    (257, 16, "laplace", 1e-10, 1, 1e-9),
    (257, 16, "cd", 1e-10, 2, 1e-9),
    (200, 16, "cd", 1e-8, 1, 1e-6),
])
def test_compressed_build_vs_oracle(dtn, n, leaf, kind, tol, level, bound):
    b, c, d = (None, None, None) if kind == "laplace" else W.cd_coeffs(n, (4101, 4102, 4103))
    op = dtn.build(n, b, c, d, leaf=leaf, tol=tol, hbs_min_level=level)
    T = op.dense()
    st = op.stats()
    op.free()
    Tref = nd_dtn(n, b, c, d, leaf=leaf)
    assert_close(T, Tref, bound, label=f"compressed n={n} {kind} tol={tol}")
    ranks = st["max_rank"]
    assert all(0 < ranks[l] < 96 for l in range(level + 1)), ranks
    assert all(ranks[l] == 0 for l in range(level + 1, len(ranks))), ranks


def test_compressed_ranks_match_pivoted_qr(dtn):
    """Level-1 W+E merge of n = 257 Laplace: the range finder's rank of S13 and S31 against the
    oracle's pivoted-QR rank at the same tolerance."""
    n, leaf, tol = 257, 16, 1e-10
    op = dtn.build(n, leaf=leaf, tol=tol, hbs_min_level=1)
    gpu_rank = op.stats()["max_rank"][1]
    op.free()
    M = assemble(n).tocsr()
    root = build_tree(n, leaf)
    sw, se = root.children[0].children[0], root.children[0].children[1]
    S1 = box_schur(M, n, sw)
    U = (sw.x0, se.x1, sw.y0, se.y1)
    ring = box_ring(sw.x0, sw.x1, sw.y0, sw.y1)
    inner = np.array([_interior_to_union(p, n, U) for p in ring])
    p1, p3 = np.nonzero(~inner)[0], np.nonzero(inner)[0]
    ref = max(pivoted_qr_rank(S1[np.ix_(p1, p3)], tol), pivoted_qr_rank(S1[np.ix_(p3, p1)], tol))
    assert abs(gpu_rank - ref) <= max(10, 0.35 * ref), (gpu_rank, ref)


def test_compressed_default_levels_closed_form(dtn):
    """n = 1100 Laplace, tol 1e-10, default rule: merges whose children's S >= 1000 (levels 0
    and 1) are compressed; the operator matches the closed form."""
    n = 1100
    op = dtn.build(n, leaf=32, tol=1e-10)
    st = op.stats()
    T = op.dense()
    op.free()
    assert_close(T, dst_dtn(n, 0.0), 1e-8, label="compressed n=1100 vs closed form")
    assert st["max_rank"][0] > 0 and st["max_rank"][1] > 0 and st["max_rank"][2] == 0, st["max_rank"]


def test_n2048_laplace_vs_closed_form(dtn):
    """The n = 2048, leaf 32 Laplace instance: the dense FP64 build and the build compressed at
    tol 1e-10 (levels 0-2) against the closed-form operator."""
    P = W.config("cfg4", "laplace")
    Tref = dst_dtn(P.n, 0.0)
    Td = dtn.build(P.n, P.b, P.c, P.d, leaf=P.leaf)
    assert_close(Td.dense(), Tref, 1e-10, label="n=2048 Laplace dense vs closed form")
    Td.free()
    Tc = dtn.build(P.n, P.b, P.c, P.d, leaf=P.leaf, tol=P.tol)
    ranks = Tc.stats()["max_rank"]
    assert_close(Tc.dense(), Tref, 1e-8, label="n=2048 Laplace compressed vs closed form")
    Tc.free()
    assert ranks[0] > 0 and max(ranks) < 96, ranks


def test_n2048_convdiff_vs_sparse_solve(dtn):
    """The n = 2048 convection-diffusion instance: four columns of T G (dense build, and compressed at
    tol 1e-10) against the oracle's sparse direct solve of the whole grid; the compressed build also
    against the dense one on 32 columns."""
    P = W.config("cfg4", "convdiff")
    Yref = np.load(os.path.join(GOLDEN, "cfg4_convdiff_Y4.npy"))
    G = P.G()[:, :32]
    Td = dtn.build(P.n, P.b, P.c, P.d, leaf=P.leaf)
    Yd = Td.apply(G)
    assert_close(Yd[:, :4], Yref, 1e-10, label="n=2048 CD dense vs sparse solve")
    Tc = dtn.build(P.n, P.b, P.c, P.d, leaf=P.leaf, tol=P.tol)
    ranks = Tc.stats()["max_rank"]
    Yc = Tc.apply(G)
    assert_close(Yc[:, :4], Yref, 1e-8, label="n=2048 CD compressed vs sparse solve")
    assert_close(Yc, Yd, 1e-8, label="n=2048 CD compressed vs dense, 32 columns")
    Tc.free()
    Td.free()
    assert ranks[0] > 0 and max(ranks) < 96, ranks


def test_rank_cap_is_an_error(dtn):
    """A tolerance no 96-column factor can certify (tol 1e-200: the residual sketch keeps every column)
    fails the build with DTN_ERANK instead of returning an operator that violates tol."""
    with pytest.raises(dtn.DtnError) as ei:
        dtn.build(257, leaf=16, tol=1e-200, hbs_min_level=1)
    assert ei.value.code == dtn.DTN_ERANK, (ei.value.code, dtn.last_error())
    assert "rank cap" in dtn.last_error()
    # the same problem at a certifiable tolerance still builds
    dtn.build(257, leaf=16, tol=1e-10, hbs_min_level=1).free()
