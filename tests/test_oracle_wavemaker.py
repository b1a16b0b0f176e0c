"""Pins of the oracle's wavemaker and sponge (Sec. 3.3; the ghost formulas
and the damping profile are readings, pinned here by what they must produce).

Expected values come from linear wave theory: a wavemaker of amplitude a
sends a progressive wave of amplitude a whose phase advances by k dx between
gauges (k from the Madsen-Sorensen relation, itself pinned elsewhere); small
waves superpose linearly, so the record of a two-component wavemaker is the
sum of the single-component records; and a sponge band absorbs the incident
wave, so the amplitude envelope along the channel is flat (a reflecting wall
instead makes a standing pattern, envelope ratio (1 + R) / (1 - R)).
"""
import math

import numpy as np
import pytest

from oracle.oracle import OracleDomain, ms_wavenumber
from paper_1909_04153_amd import scenarios as S

DEPTH, DX, NY = 0.5, 0.05, 4


def _channel(nx, bc, **kw):
    p = S.base_params(nx, NY, DX, bc=bc, wave_ramp=2.0, **kw)
    return p, np.full((NY + 1, nx + 1), DEPTH)


def _record(p, dc, gauges, t0, t1, every=5):
    """eta at the gauge cells (row 1) every `every` steps for t0 < t <= t1"""
    o = OracleDomain(p, dc)
    nx = p["nx"]
    assert o.set_state(np.zeros((NY, nx)), np.zeros((NY, nx)), np.zeros((NY, nx))) == 0
    ts, rec = [], []
    while o.info().t < t1:
        assert o.step(every) == 0
        t = o.info().t
        if t > t0:
            ts.append(t)
            rec.append(o.read("eta")[1, gauges])
    return np.array(ts), np.array(rec)


def _harmonic(ts, x, omega):
    """least-squares amplitude and phase of x(t) ~ A cos(w t) + B sin(w t) + C"""
    M = np.stack([np.cos(omega * ts), np.sin(omega * ts), np.ones_like(ts)], axis=1)
    (A, B, _), *_ = np.linalg.lstsq(M, x, rcond=None)
    return math.hypot(A, B), math.atan2(B, A)


def test_sine_wavemaker_amplitude_and_phase_speed():
    a, T = 0.004, 2.0
    w = 2.0 * math.pi / T
    k = ms_wavenumber(w, DEPTH)
    nx = 700
    p, dc = _channel(nx, (S.SINE, 0, 0, 0), wave_amp=[a], wave_omega=[w], wave_phase=[0.0])
    gauges = [int(3.0 / DX), int(4.0 / DX), int(6.0 / DX)]
    # the front (~2.1 m/s) is past the gauges by t = 10 s; the east wall's
    # reflection (35 m) is not back before t = 14 s
    ts, rec = _record(p, dc, gauges, 10.0, 14.0)
    amp, ph = zip(*(_harmonic(ts, rec[:, g], w) for g in range(len(gauges))))
    for A in amp:
        assert A == pytest.approx(a, rel=0.06)
    # eta ~ a sin(w t - k x) = A cos(w t) + B sin(w t) with atan2(B, A) =
    # pi / 2 + k x: the fitted phase grows by k (x2 - x1) downstream
    for g in range(1, len(gauges)):
        dphi = (ph[g] - ph[0]) % (2.0 * math.pi)
        expect = (k * (gauges[g] - gauges[0]) * DX) % (2.0 * math.pi)
        err = min(abs(dphi - expect), 2.0 * math.pi - abs(dphi - expect))
        assert err <= 0.05, (g, dphi, expect)


def test_two_component_wavemaker_superposes_linearly():
    comps = [(0.002, 2.0, 0.3), (0.0015, 1.4, 2.1)]   # amplitude, period, phase
    nx = 400
    gauges = [int(2.0 / DX), int(4.0 / DX)]

    def run(cs):
        p, dc = _channel(nx, (S.IRREGULAR, 0, 0, 0), wave_amp=[c[0] for c in cs],
                         wave_omega=[2.0 * math.pi / c[1] for c in cs], wave_phase=[c[2] for c in cs],
                         fixed_dt=1, dt_init=0.004)
        return _record(p, dc, gauges, 6.0, 10.0)

    ts, both = run(comps)
    _, one = run(comps[:1])
    _, two = run(comps[1:])
    scale = comps[0][0] + comps[1][0]
    # the records are of the same fixed-step times; nonlinear interaction at
    # a k ~ 0.005 is well under 5 % of the amplitude
    assert np.sqrt(np.mean((both - (one + two)) ** 2)) <= 0.05 * scale
    assert np.max(np.abs(one)) >= 0.8 * comps[0][0]
    assert np.max(np.abs(two)) >= 0.8 * comps[1][0]


def _envelope_ratio(bc_east, **kw):
    a, T = 0.003, 2.0
    w = 2.0 * math.pi / T
    nx = 400                                           # 20 m channel
    p, dc = _channel(nx, (S.SINE, bc_east, 0, 0), wave_amp=[a], wave_omega=[w], wave_phase=[0.0], **kw)
    gauges = list(range(int(6.0 / DX), int(10.0 / DX), 2))   # 4 m, about one wavelength
    ts, rec = _record(p, dc, gauges, 24.0, 30.0)
    amp = np.array([_harmonic(ts, rec[:, g], w)[0] for g in range(len(gauges))])
    return (amp.max() - amp.min()) / (amp.max() + amp.min()), amp


def test_sponge_absorbs_the_incident_wave():
    w = 2.0 * math.pi / 2.0
    L = 2.0 * math.pi / ms_wavenumber(w, DEPTH)
    r_sponge, amp = _envelope_ratio(S.SPONGE, sponge_width=(0.0, L, 0.0, 0.0), sponge_sigma=w)
    r_wall, _ = _envelope_ratio(S.WALL)
    assert r_wall > 0.5                                # a wall reflects: standing pattern
    assert r_sponge < 0.1, (r_sponge, amp)             # the sponge band: a progressive wave
    assert np.mean(amp) == pytest.approx(0.003, rel=0.15)
