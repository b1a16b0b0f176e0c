"""Tile shapes (the chunking of the line solves of Eq. 19-20 and the
stencil tile height) as a runtime choice: every candidate shape against the
oracle, a shape change in the middle of a run, and a checkpoint carried
across shapes.  A shape that raced on its LDS halo or mis-indexed a chunk
would show as an O(1) error here."""
import math

import numpy as np
import pytest

from oracle.oracle import OracleDomain
from paper_1909_04153_amd import scenarios as S

pytestmark = pytest.mark.gpu

FIELDS = ("eta", "P", "Q")
FP64_SHAPES = [(8, 16), (8, 32), (4, 16)]
FP32_SHAPES = [(16, 16), (16, 32), (8, 16), (8, 32)]


@pytest.fixture(scope="module")
def bq():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1909_04153_amd import bq as m

    m.load()
    return m


def _scales(spec):
    p = spec["params"]
    amp = max(float(np.max(np.abs(spec["eta"]))), float(np.sum(np.abs(p.get("wave_amp", [])))), 1e-3)
    c = math.sqrt(9.81 * max(float(np.max(spec["depth_c"])), 1e-3))
    return {"eta": amp, "P": amp * c, "Q": amp * c}


def _rel(a, b, s):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 0.1 * s * math.sqrt(b.size)))


CASES = {
    # 2100-cell x-lines (66..132 chunks), one-chunk y-lines
    "long_lines": lambda: S.solitary_flat(nx=2100, ny=8, dx=0.05, x0=50.0),
    # 2D, irregular wavemaker, sponges, ragged edges on both axes
    "rip_2d": lambda: S.rip_beach_scaled(98, 75, cfl=0.125, fstar_order=1, t_end=0.0),
    # wet/dry run-up under a sine wavemaker, friction, ragged sizes
    "beach_ragged": lambda: S.sloping_beach(nx=133, ny=21, dx=0.1, x_toe=1.0, amp=0.05, ramp=1.0, t_end=0.0),
    # the corrector's second pass
    "pc_hump_2d": lambda: S.closed_basin_hump(nx=70, ny=45, dx=0.1, cfl=0.25, fstar_order=2, corrector=1),
    # a last chunk of one cell on both axes in every shape (161 = 10 x 16 + 1
    # = 5 x 32 + 1, 17 = 16 + 1 = 2 x 8 + 1 = 4 x 4 + 1): the chunk solves'
    # lane groups then have empty parts
    "one_cell_chunks": lambda: S.sloping_beach(nx=161, ny=17, dx=0.1, x_toe=1.0, amp=0.05, ramp=1.0, t_end=0.0),
}


def _batch_of_one(bq, spec, precision, shape):
    g = bq.domain_from_spec(spec, precision=precision)
    b = bq.Batch([g], lanes=1)
    b.set_tune({"lanes": 1, "graph_steps": 0, "reduce_block": 256, "swizzle": 1, "reduce_segments": 1,
                "tile_y": shape[0], "chunk_x": shape[1]})
    assert (b.tune["tile_y"], b.tune["chunk_x"]) == shape
    return g, b


@pytest.mark.parametrize("shape", FP64_SHAPES)
@pytest.mark.parametrize("case", sorted(CASES))
def test_fp64_parity_in_every_tile_shape(bq, case, shape):
    spec = CASES[case]()
    o = OracleDomain(spec["params"], spec["depth_c"])
    assert o.set_state(spec["eta"], spec["P"], spec["Q"]) == 0
    g, b = _batch_of_one(bq, spec, bq.FP64, shape)
    sc = _scales(spec)
    worst = 0.0
    for k in range(8):
        assert o.step(10) == 0
        b.step(10)
        b.sync()
        for f in FIELDS:
            a, r = g.read(f), o.read(f)
            e, m = _rel(a, r, sc[f]), float(np.max(np.abs(a - r))) / sc[f]
            worst = max(worst, e)
            assert e <= 1e-12 and m <= 1e-11, (case, shape, (k + 1) * 10, f, e, m)
    print(f"{case} tile {shape[0]}x64 chunk {shape[1]} FP64 worst rel L2 {worst:.2e}")
    b.close()


@pytest.mark.parametrize("shape", FP32_SHAPES)
def test_fp32_every_tile_shape_against_the_oracle(bq, shape):
    for case in ("rip_2d", "beach_ragged", "pc_hump_2d", "one_cell_chunks"):
        spec = CASES[case]()
        o = OracleDomain(spec["params"], spec["depth_c"])
        assert o.set_state(spec["eta"], spec["P"], spec["Q"]) == 0
        g, b = _batch_of_one(bq, spec, bq.FP32, shape)
        assert o.step(200) == 0
        b.step(200)
        b.sync()
        assert g.sync().status == 0
        sc = _scales(spec)
        e = _rel(g.read("eta"), o.read("eta"), sc["eta"])
        print(f"{case} tile {shape[0]}x64 chunk {shape[1]} FP32 eta after 200 steps {e:.2e}")
        assert e <= 1e-5, (case, shape, e)
        b.close()


def test_shape_change_mid_run_and_checkpoint_across_shapes(bq):
    spec = CASES["rip_2d"]()
    o = OracleDomain(spec["params"], spec["depth_c"])
    assert o.set_state(spec["eta"], spec["P"], spec["Q"]) == 0
    g, b = _batch_of_one(bq, spec, bq.FP64, FP64_SHAPES[0])
    sc = _scales(spec)
    shapes = FP64_SHAPES + [FP64_SHAPES[0]]
    for shape in shapes:
        b.set_tune({"lanes": 1, "graph_steps": 4, "reduce_block": 256, "swizzle": 1, "reduce_segments": 1,
                    "tile_y": shape[0], "chunk_x": shape[1]})
        assert o.step(12) == 0
        b.step(12)
        b.sync()
        for f in FIELDS:
            assert _rel(g.read(f), o.read(f), sc[f]) <= 1e-12, (shape, f)
        assert abs(g.sync().t - o.info().t) <= 1e-12 * o.info().t
    # a checkpoint taken in one shape resumes in another
    blob = g.save()
    h, hb = _batch_of_one(bq, spec, bq.FP64, FP64_SHAPES[2])
    h.load_checkpoint(blob)
    assert o.step(20) == 0
    hb.step(20)
    hb.sync()
    for f in FIELDS:
        assert _rel(h.read(f), o.read(f), sc[f]) <= 1e-12, f
    b.close()
    hb.close()
