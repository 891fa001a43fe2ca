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


@pytest.mark.parametrize("n,leaf", [(3, 4), (17, 8), (100, 16), (300, 32), (301, 32), (513, 32), (1024, 32), (2048, 32)])
def test_plan_descriptors_stay_inside_their_buffers(n, leaf):
    """Host-only plan self-check: for the dense, compressed, mixed-precision and pivoted plans every
    device descriptor (products and their row/column maps, split-K partials and counters, diagonal
    blocks, interface-coupling steps, small tasks, large merges, range-finder steps) addresses only
    the buffers the plan allocates, and every launch numbers its tiles without gaps."""
    import paper_1302_5995_amd as dtn
    for tol, mixed, fast in ((0.0, False, True), (1e-10, False, True), (0.0, True, True), (0.0, False, False)):
        for sym in (False, True):
            dtn.plan_check(n, leaf, tol, mixed, fast, sym)


def test_plan_check_rejects_bad_arguments():
    import paper_1302_5995_amd as dtn
    lib = dtn.load()
    assert lib.dtn_plan_check(2, 32, 0.0, 0, 1, 0) == dtn.DTN_EINVAL
    assert lib.dtn_plan_check(64, 3, 0.0, 0, 1, 0) == dtn.DTN_EINVAL
    assert lib.dtn_plan_check(64, 8, -1.0, 0, 1, 0) == dtn.DTN_EINVAL
    assert dtn.last_error()
