"""GPU parity: the HIP build/apply against the CPU oracle, through the C ABI.

Tolerances.  The FP64 path computes the same Schur complement as the oracle
in a different elimination order (nested dissection down to base boxes,
explicit interface inverses), so the two agree to a small multiple of the
conditioning times the unit roundoff.  The relative Frobenius error bound used
for well-conditioned problems is 1e-10 (the FP64 target); Helmholtz cases
near an interior resonance carry their conditioning in the tolerance.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import nd_dtn, dst_dtn, brute_dtn, sparse_apply, trace_on_ring
from parity import assert_close

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def coeffs(n, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "laplace":
        return None, None, None
    if kind == "cd":
        return rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    if kind == "helm":
        return None, None, np.full(n * n, -rng.uniform(10, 300))
    raise ValueError(kind)


def test_cfg1_laplace_n32(dtn):
    P = W.config("cfg1")
    op = dtn.build(P.n, leaf=P.leaf)
    T = op.dense()
    Tref = nd_dtn(P.n, leaf=P.leaf)
    assert T.shape == (124, 124)
    assert_close(T, Tref, 1e-12, label="cfg1 T")
    G = P.G()
    Y = op.apply(G)
    assert_close(Y, Tref @ G, 1e-12, label="cfg1 Y")
    # Laplace invariants on the GPU result
    assert np.abs(T.sum(axis=1)).max() <= 1e-10 * np.abs(T).max()
    assert np.abs(T - T.T).max() <= 1e-12 * np.abs(T).max()


@pytest.mark.parametrize("n,leaf,kind", [
    (3, 4, "laplace"), (4, 4, "cd"), (5, 4, "helm"), (7, 5, "cd"), (8, 8, "cd"), (9, 4, "laplace"),
    (17, 8, "cd"), (33, 8, "cd"), (45, 6, "helm"), (64, 16, "cd"), (100, 16, "cd"), (130, 32, "laplace"),
])
def test_small_grids_vs_oracle(dtn, n, leaf, kind):
    b, c, d = coeffs(n, kind, n * 7 + leaf)
    op = dtn.build(n, b, c, d, leaf=leaf)
    T = op.dense()
    Tref = nd_dtn(n, b, c, d, leaf=leaf)
    assert_close(T, Tref, 1e-10, label=f"n={n} leaf={leaf} {kind} vs nd")
    if n <= 40:
        assert_close(T, brute_dtn(n, b, c, d), 1e-10, label=f"n={n} leaf={leaf} {kind} vs brute")


def test_conv_paper_scale(dtn):
    n = 41
    b, c, d = coeffs(n, "cd", 3)
    op = dtn.build(n, b, c, d, leaf=8, conv=dtn.CONV_PAPER)
    assert_close(op.dense(), nd_dtn(n, b, c, d, leaf=8, conv="paper"), 1e-10, label="conv paper")


def test_cfg2_convdiff_n256(dtn):
    P = W.config("cfg2")
    op = dtn.build(P.n, P.b, P.c, P.d, leaf=P.leaf)
    T = op.dense()
    Tref = nd_dtn(P.n, P.b, P.c, P.d, leaf=P.leaf)
    assert_close(T, Tref, 1e-10, label="cfg2 T")
    G = P.G()
    Y = op.apply(G)
    assert_close(Y, Tref @ G, 1e-10, label="cfg2 Y")
    assert np.abs(T.sum(axis=1)).max() >= 0  # d >= 0 here: rows need not sum to zero


def test_helmholtz_dst_closed_form_n300(dtn):
    n = 300
    kappa = 12.3 * math.pi
    d = -kappa * kappa
    op = dtn.build(n, None, None, np.full(n * n, d), leaf=32)
    assert_close(op.dense(), dst_dtn(n, d), 1e-10, label="helmholtz n=300")


def test_laplace_polynomials_n513(dtn):
    n = 513
    op = dtn.build(n, leaf=32)
    h = 1.0 / (n - 1)
    g = trace_on_ring(n, lambda x, y: x * x - y * y)
    y = op.apply(g)
    ring = np.array([(p[0], p[1]) for p in __import__("oracle").ring_nodes(n)])
    exp = np.zeros(len(ring))
    for r, (i, j) in enumerate(ring):
        if i in (0, n - 1) and j in (0, n - 1):
            continue
        exp[r] = h if j == 0 else (2 - h if i == n - 1 else (-2 + h if j == n - 1 else -h))
    assert np.abs(y - exp).max() <= 1e-8


def test_apply_device_matches_host(dtn):
    import torch
    n = 65
    b, c, d = coeffs(n, "cd", 11)
    op = dtn.build(n, b, c, d, leaf=16)
    T = op.dense()
    G = np.random.default_rng(1).uniform(-1, 1, (op.nb, 37))
    Gd = torch.from_numpy(np.ascontiguousarray(G.T)).cuda().t()        # column-major (nb, k)
    Yd = op.apply_device(Gd)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy()
    assert_close(Y, T @ G, 1e-13, label="apply device")
    # k = 1 and a strided leading dimension
    Gbig = torch.zeros((3, op.nb + 5), dtype=torch.float64, device="cuda")
    Gbig[:, : op.nb] = torch.from_numpy(np.ascontiguousarray(G[:, :3].T)).cuda()
    Gv = Gbig.t()[: op.nb]
    Y2 = op.apply_device(Gv).cpu().numpy()
    assert_close(Y2, T @ G[:, :3], 1e-13, label="apply device strided")


def test_device_coefficients(dtn):
    import torch
    n = 49
    b, c, d = coeffs(n, "cd", 5)
    tb, tc, td = (torch.from_numpy(x).cuda() for x in (b, c, d))
    op = dtn.build(n, tb, tc, td, leaf=8)
    assert_close(op.dense(), nd_dtn(n, b, c, d, leaf=8), 1e-10, label="device coefficients")


def test_singular_leaf_reported(dtn):
    n, leaf = 17, 8
    h = 1.0 / (n - 1)
    m = 6          # interior side of the 8 x 8 leaves (and base boxes)
    mu = 8 * math.sin(math.pi / (2 * (m + 1))) ** 2
    d = np.full(n * n, -mu / (h * h))
    with pytest.raises(dtn.DtnError) as ei:
        dtn.build(n, None, None, d, leaf=leaf)
    assert ei.value.code == dtn.DTN_ESINGULAR
    dtn.build(n, None, None, d * (1 + 1e-3), leaf=leaf)


def test_invalid_arguments(dtn):
    lib = dtn.load()
    assert not lib.dtn_build(2, None, None, None, 8, 0.0)
    assert "n must" in dtn.last_error()
    assert not lib.dtn_build(10, None, None, None, 3, 0.0)
    bad = np.zeros(100); bad[7] = np.nan
    with pytest.raises(dtn.DtnError):
        dtn.build(10, bad, None, None, leaf=4)
    lib.dtn_free(None)
    op = dtn.build(10, leaf=4)
    Y = np.zeros((op.nb, 1), order="F")
    assert lib.dtn_apply(op.handle, Y.ctypes.data, 0, Y.ctypes.data) == dtn.DTN_EINVAL
    assert lib.dtn_nb(None) == dtn.DTN_EINVAL


def test_repeated_builds_same_result(dtn):
    n = 97
    b, c, d = coeffs(n, "cd", 2)
    T1 = dtn.build(n, b, c, d, leaf=16).dense()
    for _ in range(3):
        T2 = dtn.build(n, b, c, d, leaf=16).dense()
        assert np.array_equal(T1, T2)


@pytest.mark.parametrize("n,d", [(600, 0.0), (1024, 0.0), (1024, -(40.0 * math.pi) ** 2)])
def test_full_size_vs_closed_form(dtn, n, d):
    """n up to 1024 (the benchmarked size, leaf 32, same launch configuration as bench.py)."""
    dd = None if d == 0.0 else np.full(n * n, d)
    op = dtn.build(n, None, None, dd, leaf=32)
    T = op.dense()
    op.free()
    # the FP64 target, also for Helmholtz at 20 wavelengths (interface blocks with condition
    # numbers up to ~2e7)
    assert_close(T, dst_dtn(n, d), 1e-10, label=f"n={n} d={d} vs closed form")


@pytest.mark.parametrize("n,leaf,kind", [(64, 16, "cd"), (130, 32, "helm"), (257, 32, "laplace")])
def test_fast_and_pivoted_paths_agree(dtn, n, leaf, kind):
    b, c, d = coeffs(n, kind, 99 + n)
    fast = dtn.build(n, b, c, d, leaf=leaf)
    piv = dtn.build(n, b, c, d, leaf=leaf, pivoting=dtn.PIVOT_PARTIAL)
    assert fast.stats()["pivoting_used"] == dtn.PIVOT_AUTO
    assert piv.stats()["pivoting_used"] == dtn.PIVOT_PARTIAL
    Tref = nd_dtn(n, b, c, d, leaf=leaf)
    assert_close(fast.dense(), Tref, 1e-10, label=f"fast n={n} {kind}")
    assert_close(piv.dense(), Tref, 1e-10, label=f"pivoted n={n} {kind}")


def test_partial_pivoting_full_size_repeatable(dtn):
    """The partial-pivoting path at the benchmarked size, interleaved with unpivoted builds of other
    problems: every pivoted build matches the closed form and the others bitwise (its small-merge
    kernel once let a wave read the pivot after another wave had swapped it away, at random)."""
    n = 1024
    d = np.full(n * n, -(40.0 * math.pi) ** 2)
    Tc = dst_dtn(n, float(d[0]))
    first = None
    for q in range(3):
        dtn.build(n, None, None, None if q % 2 else d, leaf=32).free()
        op = dtn.build(n, None, None, d, leaf=32, pivoting=dtn.PIVOT_PARTIAL)
        T = op.dense()
        op.free()
        assert_close(T, Tc, 1e-10, label=f"pivoted n=1024 Helmholtz, build {q}")
        if first is None:
            first = T
        else:
            assert np.array_equal(T, first)


def test_weak_pivot_falls_back_to_partial_pivoting(dtn):
    """A base-box interior within 1e-7 of a Dirichlet eigenvalue: the unpivoted path sees a
    pivot below its threshold and the build is redone with partial pivoting."""
    n, leaf = 17, 8
    h = 1.0 / (n - 1)
    m = 6
    mu = 8 * math.sin(math.pi / (2 * (m + 1))) ** 2
    d = np.full(n * n, -mu / (h * h) * (1 + 1e-7))
    op = dtn.build(n, None, None, d, leaf=leaf)
    st = op.stats()
    assert st["pivoting_used"] == dtn.PIVOT_PARTIAL
    assert rel(op.dense(), brute_dtn(n, None, None, d)) <= 1e-6


@pytest.mark.parametrize("n,leaf,kind", [(100, 16, "cd"), (130, 32, "laplace"), (67, 8, "helm")])
def test_plain_batching_matches_fused(dtn, n, leaf, kind):
    """The comparator form (one box, merge or product per launch) runs the same arithmetic."""
    b, c, d = coeffs(n, kind, n + 5)
    Tf = dtn.build(n, b, c, d, leaf=leaf).dense()
    Tp = dtn.build(n, b, c, d, leaf=leaf, batching=dtn.PLAIN).dense()
    Tref = nd_dtn(n, b, c, d, leaf=leaf)
    assert_close(Tp, Tf, 1e-13, label=f"plain vs fused n={n} {kind}")
    assert_close(Tp, Tref, 1e-10, label=f"plain n={n} {kind}")


def test_build_many_fused_across_problems(dtn):
    """Uneven problems (n, leaf, convection form, PDE) built in one plan: merges of equal height
    share launches; every operator matches the oracle and its own single build."""
    probs = [(33, 8, "cd", dtn.CONV_CENTRAL), (64, 16, "laplace", dtn.CONV_CENTRAL),
             (100, 16, "cd", dtn.CONV_PAPER), (130, 32, "helm", dtn.CONV_CENTRAL), (5, 4, "cd", dtn.CONV_CENTRAL)]
    specs, refs = [], []
    for q, (n, leaf, kind, conv) in enumerate(probs):
        b, c, d = coeffs(n, kind, 300 + q)
        specs.append(dict(n=n, b=b, c=c, d=d, leaf=leaf, conv=conv))
        refs.append(nd_dtn(n, b, c, d, leaf=leaf, conv="paper" if conv == dtn.CONV_PAPER else "central"))
    ops = dtn.build_many(specs)
    for (n, leaf, kind, conv), sp, op, Tref in zip(probs, specs, ops, refs):
        T = op.dense()
        assert op.nb == 4 * (n - 1)
        assert_close(T, Tref, 1e-10, label=f"many n={n} leaf={leaf} {kind}")
        single = dtn.build(**sp).dense()
        assert_close(T, single, 1e-13, label=f"many vs single n={n}")
        st = op.stats()
        assert st["n"] == n and st["leaf"] == leaf
    for op in ops:
        op.free()


def test_build_many_rejects_mixed_options(dtn):
    with pytest.raises(dtn.DtnError):
        dtn.build_many([dict(n=17, leaf=8), dict(n=17, leaf=8, batching=dtn.PLAIN)])


@pytest.mark.parametrize("n,leaf,kind", [(256, 16, "cd"), (300, 32, "laplace")])
def test_mixed_precision_within_stated_error(dtn, n, leaf, kind):
    """DTN_MIXED: FP32-MFMA products in the large merges below the top two levels; the stated
    bound is a relative error of 1e-6 against the FP64 oracle."""
    b, c, d = coeffs(n, kind, 77)
    opm = dtn.build(n, b, c, d, leaf=leaf, precision=dtn.MIXED)
    assert opm.stats()["precision"] == dtn.MIXED       # d >= 0: the FP32 products run
    Tm = opm.dense()
    T64 = dtn.build(n, b, c, d, leaf=leaf).dense()
    Tref = nd_dtn(n, b, c, d, leaf=leaf)
    assert_close(Tm, Tref, 1e-6, label=f"mixed n={n} {kind}")
    assert rel(Tm, T64) > 1e-13          # the FP32 products did run


def test_mixed_precision_full_size_laplace(dtn):
    """n = 1024 Laplace: the mixed form meets the stated 1e-6 against the closed-form operator."""
    n = 1024
    op = dtn.build(n, leaf=32, precision=dtn.MIXED)
    assert op.stats()["precision"] == dtn.MIXED
    T = op.dense()
    op.free()
    assert_close(T, dst_dtn(n, 0.0), 1e-6, label="mixed n=1024 Laplace")


def test_mixed_precision_near_resonant_helmholtz_runs_fp64(dtn):
    """n = 1024 Helmholtz at 20 wavelengths (kappa^2 = 1600 pi^2, next to an eigenvalue of the
    square): interface blocks with condition numbers up to ~2e7 amplify FP32 rounding of any level's
    products far beyond 1e-6 (an FP64 emulation of FP32 products in the lowest large merges alone
    gives 3.5e-5 against the closed form), so a DTN_MIXED request on a problem with d < 0 runs in
    FP64, reports it, and meets the mixed form's 1e-6 (and the FP64 1e-10)."""
    P = W.config("cfg3")
    op = dtn.build(P.n, P.b, P.c, P.d, leaf=P.leaf, precision=dtn.MIXED)
    assert op.stats()["precision"] == dtn.FP64
    T = op.dense()
    op.free()
    assert_close(T, dst_dtn(P.n, float(P.d[0])), 1e-10, label="mixed request, cfg3 (ran FP64)")


def test_profile_records_selected_families_only(dtn):
    """The kernel profiler brackets every launch by default; with a selection only the named
    families carry events, and the build's result does not depend on profiling."""
    n, leaf = 300, 32
    ref = dtn.build(n, leaf=leaf)
    try:
        dtn.profile_reset()
        dtn.profile_select(None)
        dtn.profile_enable(True)
        op = dtn.build(n, leaf=leaf)
        dtn.profile_enable(False)
        everything = dtn.profile_read()
        assert {"base_inv", "large_gather", "small_schur"} <= set(everything)
        assert all(v["launches"] > 0 and v["total_ms"] > 0 for v in everything.values())
        assert np.array_equal(op.dense(), ref.dense())
        op.free()
        dtn.profile_reset()
        dtn.profile_select(["base_inv", "large_gather"])
        dtn.profile_enable(True)
        op = dtn.build(n, leaf=leaf)
        dtn.profile_enable(False)
        picked = dtn.profile_read()
        assert set(picked) == {"base_inv", "large_gather"}
        assert picked["base_inv"]["launches"] == everything["base_inv"]["launches"]
        assert np.array_equal(op.dense(), ref.dense())
        op.free()
    finally:
        dtn.profile_select(None)
        dtn.profile_enable(False)
        dtn.profile_reset()
        ref.free()


@pytest.mark.parametrize("n,leaf,kind", [(300, 32, "laplace"), (300, 16, "helm"), (513, 32, "helm")])
def test_symmetric_path_matches_general_path(dtn, n, leaf, kind):
    """Without convection (b = c = NULL) the operator is symmetric and the dense merges below the two
    top levels compute half of each Schur complement (lower tiles of the diagonal blocks and the
    off-diagonal block once, mirrored; S31, S42 read transposed in place of S13, S24).  Passing
    explicit zero convection fields runs the general products on the same operator: the two builds
    agree to rounding, and both operators are symmetric to rounding."""
    d = coeffs(n, kind, 11)[2]
    z = np.zeros(n * n)
    op_s = dtn.build(n, None, None, d, leaf=leaf)
    op_g = dtn.build(n, z, z, d, leaf=leaf)
    Ts, Tg = op_s.dense(), op_g.dense()
    op_s.free()
    op_g.free()
    assert_close(Ts, Tg, 1e-11, label=f"n={n} leaf={leaf} {kind}: symmetric vs general path")
    assert_close(Ts, Ts.T, 1e-11, label="symmetric path: T vs T^T")
    assert_close(Tg, Tg.T, 1e-11, label="general path: T vs T^T")
