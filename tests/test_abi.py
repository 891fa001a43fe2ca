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
