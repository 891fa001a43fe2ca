"""GPU test of the allocation-free apply (dtn_apply_device_noalloc) through the C ABI.

Its split-K partial sums live in a library-owned device array instead of a workspace the handle
allocates; a column's summation order depends on nb only, so its result must be bitwise the same
as dtn_apply_device's.  Checked on two calls in a row, the second with a smaller input (fewer
columns on a smaller operator), then the wide (MFMA GEMM) case, against the oracle, and the
refusal of operators above the array's limit.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import nd_dtn
from parity import assert_close

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()      # column-major (nb, k)


def _call(dtn, fn, op, G, k):
    import torch
    Y = torch.full((k, op.nb), np.nan, dtype=torch.float64, device="cuda").t()
    # the library's stream (NULL) does not wait for torch's: finish the fill of Y first
    torch.cuda.synchronize()
    s = None
    rc = fn(op.handle, G.data_ptr(), G.stride(1) if k > 1 else op.nb, k, Y.data_ptr(),
            Y.stride(1) if k > 1 else op.nb, s)
    assert rc == dtn.DTN_OK, dtn.last_error()
    torch.cuda.synchronize()
    return Y.cpu().numpy()


@pytest.mark.parametrize("wide", [False, True])
def test_noalloc_apply_matches_apply_device(dtn, wide):
    lib = dtn.load()
    rng = np.random.default_rng(7070)
    probs = [(257, 16, 1234), (65, 8, 4321)]          # the second call: a smaller operator
    ks = [(61, 9), (200, 70)][wide]                   # and fewer columns
    for (n, leaf, seed), k in zip(probs, ks):
        r = np.random.default_rng(seed)
        b, c, d = r.uniform(-8, 8, n * n), r.uniform(-8, 8, n * n), r.uniform(0, 16, n * n)
        op = dtn.build(n, b, c, d, leaf=leaf)
        G = _dev(rng.uniform(-1, 1, (op.nb, k)))
        Yn = _call(dtn, lib.dtn_apply_device_noalloc, op, G, k)
        Yr = _call(dtn, lib.dtn_apply_device, op, G, k)
        print(f"n={n} k={k}: no-alloc vs apply_device max |diff| {np.abs(Yn - Yr).max():.3e}", flush=True)
        assert np.array_equal(Yn, Yr), (n, k)
        Tref = nd_dtn(n, b, c, d, leaf=leaf)
        assert_close(Yn, Tref @ G.cpu().numpy(), 1e-11, label=f"no-alloc n={n} k={k} vs oracle")
        op.free()


def test_noalloc_apply_full_size_and_limit(dtn):
    """n = 1024 (nb = 4092, sixteen K splits) through the Python binding, 48 and 5 columns, then the refusal of an
    operator with more ring rows than the array holds (n = 2050, nb = 8196)."""
    import torch
    lib = dtn.load()
    op = dtn.build(1024, leaf=32)
    G = _dev(np.random.default_rng(3).uniform(-1, 1, (op.nb, 48)))
    Y1 = torch.empty((48, op.nb), dtype=torch.float64, device="cuda").t()
    Y2 = torch.empty_like(Y1)
    op.apply_device(G, Y1, noalloc=True)
    op.apply_device(G, Y2)
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)
    # five columns: the narrow kernel (G read in place), whose results are those of the wide launch
    Y3 = torch.empty((5, op.nb), dtype=torch.float64, device="cuda").t()
    op.apply_device(G[:, :5], Y3, noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(Y3, Y2[:, :5])
    op.free()
    big = dtn.build(2050, leaf=32)
    Gb = torch.zeros((1, big.nb), dtype=torch.float64, device="cuda").t()
    Yb = torch.zeros_like(Gb)
    rc = lib.dtn_apply_device_noalloc(big.handle, Gb.data_ptr(), big.nb, 1, Yb.data_ptr(), big.nb, None)
    assert rc == dtn.DTN_EINVAL and "8188" in dtn.last_error()
    big.free()
