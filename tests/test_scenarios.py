"""Seeded input generators: shapes, determinism and the stated statistics."""
import math

import numpy as np

from paper_1909_04153_amd import scenarios as S


def test_shapes_and_determinism():
    for make in (lambda: S.solitary_flat(), lambda: S.sloping_beach(nx=64, ny=16),
                 lambda: S.rip_beach_scaled(128, 96), lambda: S.closed_basin_hump()):
        a, b = make(), make()
        nx, ny = a["params"]["nx"], a["params"]["ny"]
        assert a["depth_c"].shape == (ny + 1, nx + 1)
        for k in ("eta", "P", "Q"):
            assert a[k].shape == (ny, nx)
            assert np.array_equal(a[k], b[k])
        assert np.array_equal(a["depth_c"], b["depth_c"])


def test_jonswap_significant_height_and_band():
    a, om, ph = S.jonswap_components(1.0, 8.0, n=64, rng=np.random.default_rng(3))
    assert len(a) == 64
    assert abs(4.0 * math.sqrt(np.sum(a ** 2) / 2.0) - 1.0) < 1e-12
    f = om / (2 * math.pi)
    assert abs(f[0] - 0.6 / 8.0) < 1e-12 and abs(f[-1] - 2.2 / 8.0) < 1e-12
    assert np.all((ph >= 0) & (ph < 2 * math.pi))
    # the spectrum peaks near fp
    assert abs(f[np.argmax(a)] - 1.0 / 8.0) < 2 * (f[1] - f[0])


def test_rip_beach_geometry():
    s = S.rip_beach_scaled(256, 256)
    d = s["depth_c"]
    assert d[0, 0] > 7.9                      # offshore flat ~8 m
    assert d[0, -1] < 0                       # dry land at the east end
    K = len(s["rip_y"])
    assert 3 <= K <= 6
    ys = np.sort(s["rip_y"])
    assert np.all(np.diff(ys) >= 0.5 * 256 * s["params"]["dy"] / K - 1e-9)


def test_batch_mix_sizes():
    specs = S.batch_mix(64)
    assert len(specs) == 64
    cells = sum(s["params"]["nx"] * s["params"]["ny"] for s in specs)
    assert 15e6 < cells < 30e6
    for s in specs:
        assert 256 <= s["params"]["nx"] <= 1536 and 256 <= s["params"]["ny"] <= 512
