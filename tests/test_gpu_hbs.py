"""GPU tests of the HBS (telescoping) form of a built operator (Section 4) through the C ABI.

The factors are not unique (their bases depend on the random samples and the pivot order), so the
matrix they stand for and their applies are compared, never the factors: against the dense operator
the same build produced and against the oracle, at the scale of the local tolerance.  Also checked:
the memory of the factors against the dense operator and against the oracle's own HBS representation
of the same operator at the same tolerance (same tree, ranks from exact block rows), handles that keep
only the factors (every apply path and the export run the telescoping apply), and the rank cap.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import dst_dtn, nd_dtn
from oracle.hbs import hbs_compress, hbs_words, hbs_ranks
from parity import assert_close

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


@pytest.mark.parametrize("n,leaf,kind,tol", [(257, 16, "laplace", 1e-7), (257, 16, "cd", 1e-10),
                                             (130, 32, "helm", 1e-8), (33, 8, "cd", 1e-9)])
def test_hbs_reconstruction_and_apply(dtn, n, leaf, kind, tol):
    rng = np.random.default_rng(n)
    if kind == "cd":
        b, c, d = rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    elif kind == "helm":
        b, c, d = None, None, np.full(n * n, -200.0)
    else:
        b = c = d = None
    op = dtn.build(n, b, c, d, leaf=leaf)
    T = op.dense()
    info = op.hbs_compress(tol, 64)
    assert info["bytes"] > 0 and info["levels"] >= 1
    # applies through the factors against the dense operator (and the oracle's operator)
    G = rng.uniform(-1, 1, (op.nb, 40))
    Yh = op.apply_hbs_device(_dev(G)).cpu().numpy()
    assert_close(Yh, T @ G, 20 * tol, label=f"HBS apply n={n} {kind} tol={tol}")
    Tref = nd_dtn(n, b, c, d, leaf=leaf)
    assert_close(Yh, Tref @ G, 20 * tol, label=f"HBS apply vs oracle n={n}")
    # the oracle's representation of the same operator on the same tree: ranks and memory alike
    F = hbs_compress(Tref, 64, tol)
    r_gpu, r_ref = info["max_rank"], hbs_ranks(F)
    print(f"n={n} {kind} tol={tol}: ranks gpu {r_gpu} oracle {r_ref}; bytes gpu {info['bytes']} "
          f"oracle {8 * hbs_words(F)} dense {8 * op.nb ** 2}", flush=True)
    assert len(r_gpu) == len(r_ref)
    assert all(abs(a - b) <= max(6, 0.3 * b) for a, b in zip(r_gpu, r_ref)), (r_gpu, r_ref)
    assert info["bytes"] <= 1.5 * 8 * hbs_words(F)
    op.free()


def test_hbs_only_handle(dtn):
    """drop_dense: the dense T is released; dtn_apply, dtn_apply_device and dtn_export_dense run the
    telescoping apply; the allocation-free apply refuses the handle."""
    import torch
    n = 200
    rng = np.random.default_rng(5)
    b, c, d = rng.uniform(-8, 8, n * n), rng.uniform(-8, 8, n * n), rng.uniform(0, 16, n * n)
    ref = dtn.build(n, b, c, d, leaf=16)
    T = ref.dense()
    op = dtn.build(n, b, c, d, leaf=16)
    op.hbs_compress(1e-10, 48, drop_dense=True)
    st = op.stats()
    assert st["op_bytes"] == op.hbs_info()["bytes"] < T.nbytes
    Th = op.dense()
    assert_close(Th, T, 1e-9, label="HBS-only export")
    G = rng.uniform(-1, 1, (op.nb, 7))
    assert_close(op.apply(G), T @ G, 1e-9, label="HBS-only dtn_apply")
    Gd = _dev(G)
    Yd = op.apply_device(Gd).cpu().numpy()
    assert_close(Yd, T @ G, 1e-9, label="HBS-only dtn_apply_device")
    Y = torch.zeros((7, op.nb), dtype=torch.float64, device="cuda").t()
    with pytest.raises(dtn.DtnError):
        op.apply_device(Gd, Y, noalloc=True)
    op.free()
    ref.free()


def test_hbs_full_size_memory(dtn):
    """n = 1024 (the benchmark's Helmholtz operator and the Laplace operator): factors at the paper's
    local tolerance 1e-7 against the dense operator, and their memory beside the dense 134 MB (the
    paper's Table 2 reports 3.18 MB for Laplace at this size with its own construction)."""
    n = 1024
    for d in (0.0, -(40.0 * math.pi) ** 2):
        dd = None if d == 0.0 else np.full(n * n, d)
        op = dtn.build(n, None, None, dd, leaf=32)
        T = op.dense()
        info = op.hbs_compress(1e-7, 64)
        G = np.random.default_rng(1).uniform(-1, 1, (op.nb, 16))
        Yh = op.apply_hbs_device(_dev(G)).cpu().numpy()
        print(f"n=1024 d={d}: HBS {info['bytes'] / 2**20:.2f} MiB, ranks {info['max_rank']}, launches "
              f"{info['launches']}", flush=True)
        assert_close(Yh, T @ G, 2e-6, label=f"n=1024 d={d} HBS apply")
        assert info["bytes"] < 0.1 * T.nbytes
        op.free()


def test_hbs_rank_cap(dtn):
    op = dtn.build(257, leaf=16)
    with pytest.raises(dtn.DtnError) as ei:
        op.hbs_compress(1e-300, 64)
    assert ei.value.code == dtn.DTN_ERANK
    with pytest.raises(dtn.DtnError):
        op.hbs_compress(1e-7, 65)       # leaf above the limit
    info = op.hbs_compress(1e-7, 64)    # still usable
    assert info["bytes"] > 0
    op.free()
