"""The C ABI library loads and exports every symbol declared in include/bq.h
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1909_04153_amd import bq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "bq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bq_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert set(declared_symbols()) == set(bq.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(bq.LIB_PATH):
        pytest.fail("libbq.so is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(bq.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert lib.bq_abi_version() == 1


def test_workspace_size_and_parameter_checks_on_host():
    from paper_1909_04153_amd import scenarios as S

    spec = S.rip_beach_scaled(128, 64)
    n32 = bq.workspace_bytes(spec["params"], bq.FP32)
    n64 = bq.workspace_bytes(spec["params"], bq.FP64)
    assert 0 < n32 < n64
    # a wavemaker on the east side is rejected, as are tiny domains
    bad = dict(spec["params"], bc=(0, 1, 0, 0))
    with pytest.raises(bq.BqError):
        bq.workspace_bytes(bad)
    with pytest.raises(bq.BqError):
        bq.workspace_bytes(dict(spec["params"], nx=3))
