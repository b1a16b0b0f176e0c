"""The C ABI library loads and exports every symbol declared in include/bq.h
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re
import subprocess

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
    assert lib.bq_abi_version() == bq.ABI_VERSION


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


def test_domain_size_limits_on_host():
    # a square domain at the 2e9-cell limit fits the 32-bit element offsets
    # of the kernels in both precisions; an elongated one of fewer cells, whose
    # padded fields reach 2^31 elements, and one past the cell limit do not
    base = dict(nx=44721, ny=44721, dx=1.0, dy=1.0)
    for prec in (bq.FP32, bq.FP64):
        n = bq.workspace_bytes(base, prec)
        assert n > 44721 * 44721 * 4 * 15
        with pytest.raises(bq.BqError, match="32-bit offsets"):
            bq.workspace_bytes(dict(base, nx=64, ny=31_000_000), prec)
        with pytest.raises(bq.BqError, match="too large"):
            bq.workspace_bytes(dict(base, nx=44800, ny=44800), prec)


def test_binding_struct_layout_matches_the_header(tmp_path):
    """offsets and sizes of bq_params / bq_info as the C compiler lays them out"""
    fields = [f for f, _ in bq.Params._fields_]
    info = [f for f, _ in bq.Info._fields_]
    tune = [f for f, _ in bq.Tune._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "bq.h"', "int main(void) {",
           '  printf("%zu\\n", sizeof(bq_params));', '  printf("%zu\\n", sizeof(bq_info));',
           '  printf("%zu\\n", sizeof(bq_tune));']
    src += [f'  printf("%zu\\n", offsetof(bq_params, {f}));' for f in fields]
    src += [f'  printf("%zu\\n", offsetof(bq_info, {f}));' for f in info]
    src += [f'  printf("%zu\\n", offsetof(bq_tune, {f}));' for f in tune]
    src += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(bq.Params), ctypes.sizeof(bq.Info), ctypes.sizeof(bq.Tune)]
    want += [getattr(bq.Params, f).offset for f in fields] + [getattr(bq.Info, f).offset for f in info]
    want += [getattr(bq.Tune, f).offset for f in tune]
    assert got == want


def test_parameter_checks_of_the_experiment_knobs():
    from paper_1909_04153_amd import scenarios as S

    base = S.solitary_flat(64, 8)["params"]
    ts = dict(base, bc=(bq.TIMESERIES, 0, 0, 0), ts_dt=0.1, ts_eta=[0.0, 0.01], ts_P=[0.0, 0.03])
    assert bq.workspace_bytes(ts) > 0
    for bad in (dict(ts, bc=(0, bq.TIMESERIES, 0, 0)),          # east side
                dict(ts, ts_dt=0.0),                            # no spacing
                dict(base, bc=(bq.TIMESERIES, 0, 0, 0)),        # no samples
                dict(base, friction_f=-1e-3),
                dict(base, runup_delta=-0.1)):
        with pytest.raises(bq.BqError):
            bq.workspace_bytes(bad)
    with pytest.raises(ValueError):
        bq.make_params(dict(ts, ts_P=[0.0]))
    # non-finite forcing is rejected on the host
    for bad in (dict(ts, ts_eta=[0.0, float("nan")]), dict(ts, ts_P=[float("inf"), 0.0])):
        with pytest.raises(bq.BqError):
            bq.workspace_bytes(bad)
    sine = S.sloping_beach()["params"]
    assert bq.workspace_bytes(sine) > 0
    with pytest.raises(bq.BqError):
        bq.workspace_bytes(dict(sine, wave_amp=[float("nan")]))
    # the run-up record adds one interior field
    n0 = bq.workspace_bytes(base, bq.FP32)
    n1 = bq.workspace_bytes(dict(base, runup_delta=0.01), bq.FP32)
    assert n1 > n0
