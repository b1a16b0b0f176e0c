"""Transposition symmetry of the oracle's step (Sec. 2-3: the equations
treat x and y alike; Eq. 19 and 20 are the same system along the two grid
directions, and Eq. 14-15 are each other's transposes).

A state and bathymetry transposed (x <-> y, P <-> Q) must give the
transposed result.  For a flow uniform along one direction this holds bit
for bit: every cross difference then vanishes exactly, including the
four-corner cross derivatives of Eq. 12-15, which are evaluated as the
difference of two one-sided differences for that reason.  (Summed left to
right instead, the four corners leave a rounding residue on fields uniform
in x but not on fields uniform in y; the quadratic F* extrapolation then
amplifies that residue by about 2.2 per step.)  For a genuinely 2D flow the
two runs agree to rounding.
"""
import numpy as np

from oracle.oracle import OracleDomain
from paper_1909_04153_amd import scenarios as S


def _transposed(spec):
    p = dict(spec["params"])
    p["nx"], p["ny"] = spec["params"]["ny"], spec["params"]["nx"]
    p["dx"], p["dy"] = spec["params"]["dy"], spec["params"]["dx"]
    return p, spec["depth_c"].T.copy(), spec["eta"].T.copy(), spec["Q"].T.copy(), spec["P"].T.copy()


def _pair(spec):
    a = OracleDomain(spec["params"], spec["depth_c"])
    assert a.set_state(spec["eta"], spec["P"], spec["Q"]) == 0
    p, dc, eta, P, Q = _transposed(spec)
    b = OracleDomain(p, dc)
    assert b.set_state(eta, P, Q) == 0
    return a, b


def test_solitary_north_is_the_transposed_solitary_east_bit_for_bit():
    # quadratic F* extrapolation (the paper's Eq. 17), walls on all sides
    spec = S.solitary_flat(nx=400, ny=8, x0=8.0)
    a, b = _pair(spec)
    for _ in range(10):
        assert a.step(30) == 0 and b.step(30) == 0
        assert np.array_equal(a.read("eta").T, b.read("eta"))
        assert np.array_equal(a.read("P").T, b.read("Q"))
        assert np.array_equal(a.read("Q").T, b.read("P"))
        assert a.info().t == b.info().t
    # and the cross-direction flux stays exactly zero in both
    assert not np.any(a.read("Q")) and not np.any(b.read("P"))


def test_transposed_2d_hump_agrees_to_rounding():
    spec = S.closed_basin_hump(nx=70, ny=45, dx=0.1, cfl=0.125, fstar_order=1, manning_n=0.02)
    a, b = _pair(spec)
    assert a.step(300) == 0 and b.step(300) == 0
    scale = 0.05
    assert np.max(np.abs(a.read("eta").T - b.read("eta"))) < 1e-13 * scale
    for f, g in (("P", "Q"), ("Q", "P")):
        assert np.max(np.abs(a.read(f).T - b.read(g))) < 1e-13 * scale * 3.0
    assert abs(a.info().t - b.info().t) < 1e-14 * a.info().t
