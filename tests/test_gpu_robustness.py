"""Fixed versus adaptive time steps (Sec. 5.1 Fig. 5.4, Sec. 5.2 Fig. 5.7):
the study driver on a reduced conical-island basin, on the GPU."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1909_04153_amd import robustness

    return robustness


def test_adaptive_trace_and_fixed_step_bisection(rb):
    from paper_1909_04153_amd import bq

    res = rb.study(nx=151, t_end=12.0, precision=bq.FP32, snapshots=(6.0, 9.0))
    ad, fx = res["adaptive"], res["fixed"]
    print({k: v for k, v in ad.items() if k != "trace"})
    print(fx)
    assert ad["stable"], ad["reason"]
    # Eq. (47) never takes a step larger than the CFL candidate of the state
    # it starts from, so the local CFL number of the state it produces stays
    # near the target (the flow accelerates a little within one step)
    assert ad["cfl_max"] <= 0.125 * 1.1
    for s in ad["cfl_snapshots"]:
        assert s["cfl_max"] <= 0.125 * 1.1
    # the bisection brackets the largest stable fixed step to 3 %
    best = fx["largest_stable_dt"]
    assert best is not None
    unstable = [r["dt"] for r in fx["runs"] if not r["stable"]]
    assert unstable and min(unstable) <= best * 1.03 * (1 + 1e-12)
    assert all(r["stable"] for r in fx["runs"] if r["dt"] <= best)
    # the wave climbed the island's west face above the still-water line
    radii = ad["runup_over_shoreline_radius"]
    west = radii[len(radii) // 2 - 1: len(radii) // 2 + 1]
    assert min(west) < 1.0


def test_rip_beach_study_runs_without_an_island(rb):
    # the study driver on the rip beach under irregular waves (Sec. 5.4,
    # Fig. 5.18) at 128 x 128 cells of 8 m over 60 s: the adaptive run holds
    # the CFL target, the bisection brackets the largest stable fixed step,
    # and no run-up radii are reported (the beach has no island)
    from paper_1909_04153_amd import bq

    res = rb.study(nx=128, t_end=60.0, precision=bq.FP32, snapshots=(20.0, 40.0), scenario="rip")
    ad, fx = res["adaptive"], res["fixed"]
    print({k: v for k, v in ad.items() if k != "trace"})
    print(fx)
    assert ad["stable"], ad["reason"]
    assert ad["cfl_max"] <= 0.125 * 1.1
    best = fx["largest_stable_dt"]
    assert best is not None
    unstable = [r["dt"] for r in fx["runs"] if not r["stable"]]
    assert unstable and min(unstable) <= best * 1.03 * (1 + 1e-12)
    assert ad["runup_over_shoreline_radius"] is None
