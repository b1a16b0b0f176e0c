"""Release of library-created HIP objects, and FP32 friction on a bed whose
still-water depth is exactly zero (through the C ABI)."""
import math

import numpy as np
import pytest

from oracle.oracle import OracleDomain
from paper_1909_04153_amd import scenarios as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bq():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1909_04153_amd import bq as m

    m.load()
    return m


def test_batch_free_releases_streams_events_and_graphs(bq):
    # four-lane batches with graph replays and event-timed profiles, created
    # and freed repeatedly: every stream, event and graph executable the
    # library made for them is destroyed again
    specs = [S.sloping_beach(nx=96, ny=40, dx=0.1, x_toe=2.0, t_end=0.0),
             S.solitary_flat(nx=70, ny=20, x0=1.0),
             S.closed_basin_hump(nx=40, ny=30, dx=0.1, cfl=0.125, fstar_order=1),
             S.rip_beach_scaled(64, 48, cfl=0.125, fstar_order=1, t_end=0.0)]
    doms = [bq.domain_from_spec(s, precision=bq.FP32) for s in specs]
    for d in doms:
        d.set_graph_steps(4)
        d.step(8)
        d.sync()
    base = bq.live_handles()
    for rep in range(6):
        b = bq.Batch(doms, lanes=4)
        assert b.lanes == 4
        b.set_graph_steps(4)
        b.step(8)
        b.profile(1)
        b.set_lanes(2)
        b.step(8)
        b.close()
        assert bq.live_handles() == base, (rep, bq.live_handles(), base)
    for d in doms:
        d.close()
    after = bq.live_handles()
    assert after["graphs"] == base["graphs"] - len(doms)
    assert after["streams"] == base["streams"] and after["events"] == base["events"]


def test_fp32_manning_friction_on_a_dry_bed_at_the_still_water_line(bq):
    # Ritter dam break over a bed at the still-water level (d = 0 everywhere)
    # with Manning friction: cells ahead of the front hold films whose depth
    # can be FP32-subnormal, where h^(-1/3) must stay finite.  FP32 against
    # the FP64 oracle: the dry front amplifies a rounding-level difference
    # about a thousandfold (the oracle against itself, pinned in
    # test_oracle_physics.py), so FP32's 6e-8 rounding is held to 1e-3.
    spec = S.dam_break_dry_bed(nx=150, ny=6, dx=0.1, manning_n=0.015)
    o = OracleDomain(spec["params"], spec["depth_c"])
    assert o.set_state(spec["eta"], spec["P"], spec["Q"]) == 0
    g = bq.domain_from_spec(spec, precision=bq.FP32)
    assert o.step(200) == 0
    g.step(200)
    gi = g.sync()
    assert gi.status == 0 and gi.n == 200, gi
    eta_g, eta_o = g.read("eta"), o.read("eta")
    assert np.all(np.isfinite(eta_g)) and np.all(np.isfinite(g.read("P")))
    err = float(np.linalg.norm(eta_g - eta_o) / np.linalg.norm(eta_o))
    print(f"dam break with Manning friction FP32 after 200 steps: eta rel L2 {err:.2e}")
    assert err <= 1e-3
