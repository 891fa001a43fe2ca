"""C-ABI contract checks that need no GPU: the library loads and exports every symbol
include/dtn.h declares, and calls fail cleanly (no crash) when no device is present."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "dtn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(dtn_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_symbols()
    for s in ("dtn_build", "dtn_apply", "dtn_free", "dtn_build_ex", "dtn_apply_device", "dtn_build_many"):
        assert s in names


def test_library_exports_every_declared_symbol():
    import paper_1302_5995_amd as dtn
    lib = dtn.load()
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert set(declared_symbols()) <= set(dtn.EXPORTS)


def test_calls_fail_cleanly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1302_5995_amd as dtn
    lib = dtn.load()
    assert not lib.dtn_build(16, None, None, None, 8, 0.0)
    assert dtn.last_error()
    assert lib.dtn_nb(None) == dtn.DTN_EINVAL
    lib.dtn_free(None)
    assert dtn.version().startswith("dtn")


def test_import_dense_rejects_bad_arguments():
    """dtn_import_dense checks its arguments before touching a device: NULL with a message."""
    import ctypes
    import numpy as np
    import paper_1302_5995_amd as dtn
    lib = dtn.load()
    T = np.zeros((4, 4), order="F")
    assert not lib.dtn_import_dense(0, T.ctypes.data, 4, 0)           # nb < 1
    assert "nb" in dtn.last_error()
    assert not lib.dtn_import_dense(4, None, 4, 0)                     # no matrix
    assert not lib.dtn_import_dense(4, T.ctypes.data, 3, 0)            # ldt < nb
    assert "ldt" in dtn.last_error()
    with pytest.raises(ValueError):
        dtn.import_dense(np.zeros((3, 4)))                             # not square


@pytest.mark.parametrize("n,leaf", [(3, 4), (17, 8), (100, 16), (300, 32), (301, 32), (513, 32), (1024, 32), (2048, 32)])
def test_plan_descriptors_stay_inside_their_buffers(n, leaf):
    """Host-only plan self-check: for the dense, compressed, mixed-precision and pivoted plans every
    device descriptor (products and their row/column maps, split-K partials and counters, diagonal
    blocks, interface-coupling steps, small tasks, large merges, range-finder steps) addresses only
    the buffers the plan allocates, and every launch numbers its tiles without gaps."""
    import paper_1302_5995_amd as dtn
    for tol, mixed, fast in ((0.0, False, True), (1e-10, False, True), (0.0, True, True), (0.0, False, False)):
        for sym in (0, 1, 2):
            dtn.plan_check(n, leaf, tol, mixed, fast, sym)


def test_plan_check_rejects_bad_arguments():
    import paper_1302_5995_amd as dtn
    lib = dtn.load()
    assert lib.dtn_plan_check(2, 32, 0.0, 0, 1, 0) == dtn.DTN_EINVAL
    assert lib.dtn_plan_check(64, 3, 0.0, 0, 1, 0) == dtn.DTN_EINVAL
    assert lib.dtn_plan_check(64, 8, -1.0, 0, 1, 0) == dtn.DTN_EINVAL
    assert dtn.last_error()


def test_plan_footprint_keys_follow_the_plan_cache():
    """Serving admission charges each plan once per plan-cache key.  Builds of one n and leaf with and
    without convection run on different plans (the symmetric one mirrors its Schur products), as do
    mixed-precision and compressed builds: each gets its own key and is charged separately; the
    unpivoted build also carries the partial-pivoting plan it may fall back to.  (Plans already cached
    in the process count zero, so the size is one no other test builds.)"""
    import numpy as np
    import paper_1302_5995_amd as dtn
    n = 71
    z = np.zeros(n * n)
    sym_b, sym_k = dtn.plan_footprint(n, leaf=16)
    gen_b, gen_k = dtn.plan_footprint(n, z, z, None, leaf=16)
    mix_b, mix_k = dtn.plan_footprint(n, leaf=16, precision=dtn.MIXED)
    cmp_b, cmp_k = dtn.plan_footprint(n, leaf=16, tol=1e-10, hbs_min_level=1)
    piv_b, piv_k = dtn.plan_footprint(n, leaf=16, pivoting=dtn.PIVOT_PARTIAL)
    assert len({sym_k, gen_k, mix_k, cmp_k, piv_k}) == 5
    assert min(sym_b, gen_b, mix_b, cmp_b, piv_b) > 0
    # the unpivoted plan is charged with its pivoted fallback
    assert sym_b > piv_b
    # the workspaces hold at least the level buffers: two levels of four 35 x 35 boxes' Schur complements
    assert piv_b >= 8 * 4 * (4 * 34) ** 2
    lib = dtn.load()
    import ctypes as C
    assert lib.dtn_plan_footprint(None, None, None, 0) == dtn.DTN_EINVAL
    D, keep = dtn.make_desc(2, leaf=16)
    nb = C.c_size_t(0)
    assert lib.dtn_plan_footprint(C.byref(D), C.byref(nb), None, 0) == dtn.DTN_EINVAL


@pytest.mark.parametrize("n,leaf", [(17, 8), (300, 32), (1024, 32), (2048, 32)])
def test_plan_descriptors_stay_inside_their_buffers_under_any_tile(n, leaf):
    """The autotuner may give any product launch any tile it can take: the plan stays in bounds
    for each forced tile (64 x 64, 128 x 128, 32 x 32, 32 x 32 with deep K chunks)."""
    import paper_1302_5995_amd as dtn
    for tile in (0, 2, 3, 4):
        for tol, sym in ((0.0, 0), (0.0, 2), (1e-10, 0)):
            dtn.plan_check_tiles(n, leaf, tol, False, True, sym, tile)


def test_tune_cache_json_round_trip(tmp_path):
    """The tuning table's JSON cache: written, read back, refused when written for another
    architecture or malformed (host-only; the table starts empty in this process)."""
    import paper_1302_5995_amd as dtn
    dtn.tune_clear()
    good = tmp_path / "tune.json"
    good.write_text('{"arch": "gfx950", "tiles": {"d3t1056M2046N2046K1022a0e1s0b1f1": 2, "d1t16M64N64K64a0e0s0b0f1": 3}}')
    dtn.tune_load(str(good))
    assert dtn.tune_size() == 2
    out = tmp_path / "out.json"
    dtn.tune_save(str(out))
    import json
    back = json.loads(out.read_text())
    assert back["arch"] == "gfx950" and back["tiles"]["d1t16M64N64K64a0e0s0b0f1"] == 3
    for bad in ('{"arch": "gfx942", "tiles": {}}', '{"arch": "gfx950", "tiles": {"x": 7}}', '{"arch": "gfx950"',
                '[1, 2]'):
        p = tmp_path / "bad.json"
        p.write_text(bad)
        with pytest.raises(dtn.DtnError):
            dtn.tune_load(str(p))
    with pytest.raises(dtn.DtnError):
        dtn.tune_load(str(tmp_path / "missing.json"))
    dtn.tune_clear()
    assert dtn.tune_size() == 0


@pytest.mark.parametrize("n,leaf,fast,sym", [(33, 8, True, 0), (65, 16, True, 1), (65, 16, False, 0),
                                              (129, 32, True, 2), (257, 32, False, 1), (300, 32, True, 0)])
def test_body_plan_stays_inside_its_buffers(n, leaf, fast, sym):
    """Host-only: the body-load updates of random loads (plus loads on box rings and next to the grid's
    ring) for the fast and partially pivoted plans: every gather, inversion and product in bounds."""
    import numpy as np
    import paper_1302_5995_amd as dtn
    rng = np.random.default_rng(n)
    pts = {(int(rng.integers(1, n - 1)), int(rng.integers(1, n - 1))) for _ in range(40)}
    pts |= {(1, 1), (n - 2, n - 2), (leaf - 1, leaf), (n // 2, n // 2)}
    dtn.body_plan_check(n, sorted(pts), leaf=leaf, fast=fast, sym=sym)
    dtn.body_plan_check(n, [(n // 3, n // 4)], leaf=leaf, fast=fast, sym=sym)


def test_body_plan_rejects_bad_nodes():
    import paper_1302_5995_amd as dtn
    with pytest.raises(dtn.DtnError):
        dtn.body_plan_check(33, [(0, 5)], leaf=8)        # a ring node
    with pytest.raises(dtn.DtnError):
        dtn.body_plan_check(33, [(4, 5), (4, 5)], leaf=8)   # listed twice
