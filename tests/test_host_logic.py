"""Host-side logic that needs no GPU: the study driver's bisection and
run-up measure, the serving loop's bookkeeping, the scenario generators of
the experiment knobs."""
import math

import numpy as np
import pytest

from paper_1909_04153_amd import robustness as R
from paper_1909_04153_amd import scenarios as S


def test_bisection_brackets_the_threshold(monkeypatch):
    # a fake run that is stable exactly below dt* = 0.0123
    calls = []

    class FakeDomain:
        def close(self):
            pass

    def fake_run(spec, t_end, precision, fixed_dt=None, every=64):
        calls.append(fixed_dt)
        ok = fixed_dt < 0.0123
        return dict(stable=ok, steps=int(t_end / fixed_dt), reason="ok" if ok else "NaN", domain=FakeDomain())

    monkeypatch.setattr(R, "run", fake_run)
    best, runs = R.largest_stable_fixed_dt({}, 1.0, 1e-4, 0.1, rel_tol=0.01)
    assert best < 0.0123 <= best * 1.01 * (1 + 1e-12)
    assert min(dt for dt, st, _, _ in runs if not st) <= best * 1.01 * (1 + 1e-12)
    # a stable upper bound or an unstable lower bound ends the search at once
    best, _ = R.largest_stable_fixed_dt({}, 1.0, 1e-4, 0.01)
    assert best == 0.01
    best, _ = R.largest_stable_fixed_dt({}, 1.0, 0.02, 0.1)
    assert best is None


def test_runup_radii_of_a_synthetic_record():
    # inundation of the island's land cells down to radius r_in on the west
    # half only: the west sectors report r_in / R, the east ones 1 (no land
    # cell inundated there)
    spec = S.conical_island(nx=121, ny=121, dx=0.25)
    nx, ny, dx = 121, 121, 0.25
    X, Y = S.cell_coords(nx, ny, dx, dx)
    xc, yc = spec["center"]
    r = np.hypot(X - xc, Y - yc)
    r_in = 1.6
    rec = np.where((r >= r_in) & (X < xc), 0.1, np.nan)
    radii = R.runup_radii(spec, rec, n_dir=8)
    R0 = spec["shore_radius"]
    west = radii[3:5]            # sectors around angle pi
    east = [radii[0], radii[7]]
    assert all(abs(v - r_in / R0) < 0.25 / R0 for v in west)
    assert all(v == 1.0 for v in east)


def test_series_beach_and_island_generators():
    s = S.series_beach(nx=64, ny=8, dx=0.05)
    p = s["params"]
    assert p["bc"][0] == S.TIMESERIES and len(p["ts_eta"]) == len(p["ts_P"]) > 100
    assert p["runup_delta"] == pytest.approx(0.1 * 0.05 / 3.0)
    assert np.allclose(np.array(p["ts_P"]), math.sqrt(9.81 * 0.4) * np.array(p["ts_eta"]))
    c = S.conical_island(nx=121, ny=121, dx=0.25)
    assert c["shore_radius"] == pytest.approx(2.32)
    # the island top is 0.305 m above still water; the basin floor 0.32 m deep
    assert c["depth_c"].min() == pytest.approx(-0.305) and c["depth_c"].max() == pytest.approx(0.32)
    # the solitary wave starts west of the island, clear of it
    X, _ = S.cell_coords(121, 121, 0.25, 0.25)
    assert X[c["eta"] > 1e-3].max() < c["center"][0] - 3.6
