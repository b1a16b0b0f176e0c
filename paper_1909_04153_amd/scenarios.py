"""Seeded synthetic scenarios: bathymetry, initial states and wave forcing.

This module only generates inputs (shapes, sizes, value distributions); it
contains none of the solver's arithmetic.  Both the GPU library and the CPU
oracle consume what it produces, so it is the one piece they share.

The paper's laboratory benchmarks (conical island, Lynett et al. 2019 shelf,
Haller et al. 2002 and Hamm 1992 rip-channel basins, Sec. 5) are not available
here; the generators below stand in for them with the same kinds of geometry
and forcing: a solitary wave on a flat bed, a plane beach running up to dry
land under a sine wavemaker, a barred beach cut by rip channels under a
JONSWAP irregular wavemaker with sponge side walls, and seeded mixtures of
these for batched and served runs.

A scenario is a plain dict ``spec`` with keys
  params   -- solver parameters (nx, ny, dx, dy, B, manning_n, cfl, bc, ...)
  depth_c  -- (ny+1, nx+1) still-water depth at cell corners (+wet, -land)
  eta, P, Q -- (ny, nx) initial state (eta = h - d)
  steps / t_end -- run length
"""
from __future__ import annotations

import math

import numpy as np

G = 9.81
B_MS = 1.0 / 15.0
WALL, SINE, SPONGE, IRREGULAR, TIMESERIES = 0, 1, 2, 3, 4


def base_params(nx, ny, dx, dy=None, **kw):
    p = dict(nx=int(nx), ny=int(ny), dx=float(dx), dy=float(dy if dy is not None else dx), g=G, B=B_MS,
             manning_n=0.0, cfl=0.2, ema_alpha=0.1, dt_init=0.0, dt_max=1.0, dt_min=1e-9, fixed_dt=0,
             theta=1.3, eps_desing=0.0, bc=(WALL, WALL, WALL, WALL), sponge_width=(0.0, 0.0, 0.0, 0.0),
             sponge_sigma=0.0, wave_amp=[], wave_omega=[], wave_phase=[], wave_ramp=0.0, t_end=0.0,
             fstar_order=2, friction_f=0.0, runup_delta=0.0)
    p.update(kw)
    return p


def corner_coords(nx, ny, dx, dy):
    x = np.arange(nx + 1) * dx
    y = np.arange(ny + 1) * dy
    return np.meshgrid(x, y)  # (ny+1, nx+1)


def cell_coords(nx, ny, dx, dy):
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    return np.meshgrid(x, y)  # (ny, nx)


def rest_state(nx, ny):
    z = np.zeros((ny, nx))
    return z, z.copy(), z.copy()


def solitary_profile(x, x0, a, d):
    """Initial-condition profile a sech^2(k (x - x0)) with k = sqrt(3a / 4d^3)
    and the flux c * eta, c = sqrt(g (d + a)) (Boussinesq-type solitary wave)."""
    k = math.sqrt(3.0 * a / (4.0 * d ** 3))
    eta = a / np.cosh(k * (x - x0)) ** 2
    c = math.sqrt(G * (d + a))
    return eta, c * eta


# ---------------------------------------------------------------------------
# C1: solitary wave on a flat bed (plain method, FP64)
# ---------------------------------------------------------------------------

def solitary_flat(nx=200, ny=20, dx=0.05, depth=1.0, amp=0.1, x0=3.0, steps=300, **kw):
    p = base_params(nx, ny, dx, **kw)
    depth_c = np.full((ny + 1, nx + 1), float(depth))
    X, _ = cell_coords(nx, ny, dx, p["dy"])
    eta, P = solitary_profile(X, x0, amp, depth)
    return dict(name=f"solitary_flat_{nx}x{ny}", params=p, depth_c=depth_c, eta=eta, P=P,
                Q=np.zeros_like(eta), steps=steps)


# ---------------------------------------------------------------------------
# C2: plane beach up to dry land, sine wavemaker, Manning friction
# ---------------------------------------------------------------------------

def sloping_beach(nx=1024, ny=256, dx=0.1, h_off=0.5, x_toe=10.0, slope=1.0 / 20.0, amp=0.02, period=2.0,
                  ramp=4.0, manning=0.015, t_end=20.0, **kw):
    """Flat offshore depth h_off for x < x_toe, then a 1:(1/slope) beach that
    crosses the still-water line at x_toe + h_off / slope and continues as
    dry land; sine wavemaker on the west side, walls elsewhere."""
    p = base_params(nx, ny, dx, manning_n=manning, bc=(SINE, WALL, WALL, WALL), wave_amp=[amp],
                    wave_omega=[2.0 * math.pi / period], wave_phase=[0.0], wave_ramp=ramp, **kw)
    Xc, _ = corner_coords(nx, ny, dx, p["dy"])
    b = np.where(Xc < x_toe, -h_off, -h_off + (Xc - x_toe) * slope)
    eta, P, Q = rest_state(nx, ny)
    return dict(name=f"sloping_beach_{nx}x{ny}", params=p, depth_c=-b, eta=eta, P=P, Q=Q, t_end=t_end)


# ---------------------------------------------------------------------------
# C3: barred beach with seeded rip channels, JONSWAP irregular waves
# ---------------------------------------------------------------------------

def jonswap_components(hs, tp, gamma=3.3, n=64, fmin_ratio=0.6, fmax_ratio=2.2, rng=None):
    """n equal-df components of a JONSWAP spectrum on [fmin, fmax] * fp with
    amplitudes sqrt(2 S df) scaled so that 4 sqrt(m0) = Hs, random phases."""
    fp = 1.0 / tp
    f = np.linspace(fmin_ratio * fp, fmax_ratio * fp, n)
    df = f[1] - f[0]
    sig = np.where(f <= fp, 0.07, 0.09)
    r = np.exp(-((f - fp) ** 2) / (2.0 * sig ** 2 * fp ** 2))
    S = G ** 2 * (2.0 * math.pi) ** -4 * f ** -5 * np.exp(-1.25 * (fp / f) ** 4) * gamma ** r
    a = np.sqrt(2.0 * S * df)
    m0 = np.sum(a ** 2) / 2.0
    a *= hs / (4.0 * math.sqrt(m0))
    rng = rng if rng is not None else np.random.default_rng(0)
    phase = rng.uniform(0.0, 2.0 * math.pi, n)
    return a, 2.0 * math.pi * f, phase


def rip_beach(nx=2048, ny=2048, dx=0.5, seed=190904153, hs=1.0, tp=8.0, gamma=3.3, n_waves=64,
              sponge=48.0, manning=0.015, t_end=600.0, h_off=8.0, x_toe=300.0, x_shore=780.0,
              bar_x=660.0, bar_amp=1.0, bar_sigma=20.0, **kw):
    rng = np.random.default_rng(seed)
    Ly = ny * dx
    # rip channels: K ~ U{3..6} at jittered, evenly spread alongshore
    # positions (spacing at least Ly / (2K))
    K = int(rng.integers(3, 7))
    ys = [float((k + 0.5 + rng.uniform(-0.25, 0.25)) * Ly / K) for k in range(K)]
    sig_y = rng.uniform(15.0, 30.0, K) * min(1.0, Ly / 1024.0)
    a, om, ph = jonswap_components(hs, tp, gamma, n_waves, rng=rng)
    p = base_params(nx, ny, dx, manning_n=manning, bc=(IRREGULAR, WALL, SPONGE, SPONGE),
                    sponge_width=(0.0, 0.0, sponge, sponge), sponge_sigma=2.0 * math.pi / tp,
                    wave_amp=list(a), wave_omega=list(om), wave_phase=list(ph), wave_ramp=2.0 * tp, **kw)
    Xc, Yc = corner_coords(nx, ny, dx, p["dy"])
    slope = h_off / (x_shore - x_toe)
    b = np.where(Xc < x_toe, -h_off, -h_off + (Xc - x_toe) * slope)
    cut = np.ones_like(Yc)
    for yk, sk in zip(ys, sig_y):
        cut *= 1.0 - np.exp(-(((Yc - yk) / sk) ** 2))
    b = b + bar_amp * np.exp(-((Xc - bar_x) ** 2) / (2.0 * bar_sigma ** 2)) * cut
    eta, P, Q = rest_state(nx, ny)
    return dict(name=f"rip_beach_{nx}x{ny}", params=p, depth_c=-b, eta=eta, P=P, Q=Q, t_end=t_end,
                rip_y=ys)


def series_beach(nx=256, ny=32, dx=0.05, h_off=0.4, x_toe=2.0, slope=0.1, hs=0.04, tp=1.2, n_waves=16,
                 ts_dt=0.02, duration=120.0, friction_f=0.0025, seed=190904156, ramp=2.0, **kw):
    """Plane beach driven by a time-series boundary with the knobs of the
    paper's experiments (Sec. 3.3, 5.1, 5.3-5.4): the west boundary follows a
    seeded JONSWAP surface record eta(t) = sum a_m sin(w_m t + p_m) sampled
    every ts_dt, with the long-wave flux P = sqrt(g h_off) eta; quadratic
    friction factor f; run-up record with threshold s dx / 3."""
    rng = np.random.default_rng(seed)
    a, om, ph = jonswap_components(hs, tp, 3.3, n_waves, rng=rng)
    t = np.arange(int(round(duration / ts_dt)) + 1) * ts_dt
    eta_t = np.sum(a[:, None] * np.sin(om[:, None] * t[None, :] + ph[:, None]), axis=0)
    p = base_params(nx, ny, dx, bc=(TIMESERIES, WALL, WALL, WALL), ts_dt=ts_dt, ts_eta=list(eta_t),
                    ts_P=list(math.sqrt(G * h_off) * eta_t), wave_ramp=ramp, friction_f=friction_f,
                    runup_delta=slope * dx / 3.0, **kw)
    Xc, _ = corner_coords(nx, ny, dx, p["dy"])
    b = np.where(Xc < x_toe, -h_off, -h_off + (Xc - x_toe) * slope)
    eta, P, Q = rest_state(nx, ny)
    return dict(name=f"series_beach_{nx}x{ny}", params=p, depth_c=-b, eta=eta, P=P, Q=Q)


def conical_island(nx=601, ny=601, dx=0.05, depth=0.32, rel_height=0.18, r_top=1.1, island_h=0.625,
                   island_slope=0.25, x0=5.0, sponge=2.0, sponge_sigma=5.0, **kw):
    """Stand-in for the conical-island run-up test (Sec. 5.1): a square basin
    of nx x ny cells of dx (30 m at the defaults) and depth 0.32 m with a
    conical island at its centre (top diameter 2.2 m, side slope 1:4, 0.625 m
    high, so 7.2 m across at the base and a still-water shoreline radius of
    2.32 m); a solitary wave of height 0.18 d starts at x0 near the west
    side; sponge layers west and east, walls north and south, no friction.
    2D dispersive case: CFL 0.125 and linear F* extrapolation.  The run-up
    record uses the paper's threshold s dx / 3."""
    kw.setdefault("cfl", 0.125)
    kw.setdefault("fstar_order", 1)
    p = base_params(nx, ny, dx, bc=(SPONGE, SPONGE, WALL, WALL), sponge_width=(sponge, sponge, 0.0, 0.0),
                    sponge_sigma=sponge_sigma, runup_delta=island_slope * dx / 3.0, **kw)
    Xc, Yc = corner_coords(nx, ny, dx, p["dy"])
    xc, yc = 0.5 * nx * dx, 0.5 * ny * p["dy"]
    r = np.hypot(Xc - xc, Yc - yc)
    top = -depth + island_h
    b = np.minimum(top, -depth + np.maximum(island_h - (r - r_top) * island_slope, 0.0))
    X, _ = cell_coords(nx, ny, dx, p["dy"])
    eta, P = solitary_profile(X, x0, rel_height * depth, depth)
    return dict(name=f"conical_island_{nx}x{ny}", params=p, depth_c=-b, eta=eta, P=P, Q=np.zeros_like(eta),
                center=(xc, yc), shore_radius=r_top + (island_h - depth) / island_slope)


def airy_wavenumber(omega, h):
    """Wave number of linear (Airy) theory, omega^2 = g k tanh(k h), by Newton
    iteration on a table of depths interpolated to the given ones (used only
    to lay a plausible wave field over an initial state; the solver's own
    relation is not used here)."""
    h = np.maximum(np.asarray(h, dtype=np.float64), 1e-3)
    tab = np.geomspace(1e-3, max(float(np.max(h)), 2e-3), 4096)
    k = omega / np.sqrt(G * tab)
    for _ in range(40):
        t = np.tanh(k * tab)
        f = G * k * t - omega * omega
        df = G * t + G * k * tab * (1.0 - t * t)
        k = k - f / df
    return np.interp(h, tab, k)


def spun_up(spec, h_taper=(0.3, 0.1), ramp_off=True):
    """The scenario with its west wavemaker's wave train already in the
    domain at t = 0: eta = A sum_m a_m sin(phi_m - theta_m), theta_m the
    integral along x of the local Airy wave number of component m, flux
    P = (omega_m / k_m) eta_m (waves travelling east), Q = 0.  The envelope A
    falls from 1 to 0 (sin^2) where the still-water depth drops from
    h_taper[0] to h_taper[1] (relative to the offshore depth), so the train
    stops short of the shoreline.  ramp_off: no start-up ramp, so the
    wavemaker's values continue the field at the boundary."""
    out = dict(spec)
    p = dict(spec["params"])
    if ramp_off:
        p["wave_ramp"] = 0.0
    out["params"] = p
    nx, ny, dx = p["nx"], p["ny"], p["dx"]
    dc = spec["depth_c"]
    dcell = 0.25 * (dc[:-1, :-1] + dc[1:, :-1] + dc[:-1, 1:] + dc[1:, 1:])
    h0 = float(np.max(dcell[:, 0]))
    z = np.clip((dcell / h0 - h_taper[1]) / (h_taper[0] - h_taper[1]), 0.0, 1.0)
    # the envelope also stays 0 beyond the first cell that falls below the
    # taper's lower end, so no wave is laid behind a bar or on land
    blocked = np.cumsum(dcell / h0 <= h_taper[1], axis=1) > 0
    A = np.where(blocked, 0.0, np.sin(0.5 * math.pi * z) ** 2)
    eta = np.zeros((ny, nx))
    P = np.zeros((ny, nx))
    amps, oms = p.get("wave_amp", []), p.get("wave_omega", [])
    phs = p.get("wave_phase", [0.0] * len(amps))
    for a, om, ph in zip(amps, oms, phs):
        k = airy_wavenumber(om, dcell)
        theta = np.cumsum(k, axis=1) * dx - 0.5 * k * dx   # integral to the cell centre
        e = a * A * np.sin(ph - theta)
        eta += e
        P += (om / k) * e
    out["eta"], out["P"], out["Q"] = eta, P, np.zeros_like(eta)
    out["name"] = spec["name"] + "_spun_up"
    return out


def transposed_solitary(nx=64, ny=1536, dx=0.05, depth=1.0, amp=0.1, y0=8.0, **kw):
    """C1's solitary wave travelling north along a channel of ny cells: the
    y-lines carry the wave (many chunks per line)."""
    p = base_params(nx, ny, dx, **kw)
    depth_c = np.full((ny + 1, nx + 1), float(depth))
    _, Y = cell_coords(nx, ny, dx, p["dy"])
    eta, Q = solitary_profile(Y, y0, amp, depth)
    return dict(name=f"solitary_north_{nx}x{ny}", params=p, depth_c=depth_c, eta=eta, P=np.zeros_like(eta),
                Q=Q)


def shelf_breaking(nx=400, ny=80, dx=0.1, h_off=0.78, x_toe=10.0, slope=1.0 / 15.0, h_shelf=0.05,
                   rel_height=0.5, x0=5.0, island_x=28.0, island_r=1.0, island_h=0.25, island_slope=0.25,
                   manning=0.0, **kw):
    """Stand-in for the breaking solitary wave over a shelf (Sec. 5.2, the
    Lynett et al. 2019 experiment, whose gauge data are not available): a
    flat offshore region of depth h_off, a 1:15 slope up to a shallow shelf
    of still-water depth h_shelf that runs to the east wall, a conical island
    on the shelf (top above still water), and a solitary wave of height
    rel_height * h_off starting at x0, so that it steepens and breaks on the
    slope and crosses the shelf as a bore; sponge west, walls elsewhere.
    2D dispersive case: CFL 0.125, linear F* extrapolation."""
    kw.setdefault("cfl", 0.125)
    kw.setdefault("fstar_order", 1)
    p = base_params(nx, ny, dx, bc=(SPONGE, WALL, WALL, WALL), sponge_width=(3.0, 0.0, 0.0, 0.0),
                    sponge_sigma=2.0, manning_n=manning, runup_delta=slope * dx / 3.0, **kw)
    Xc, Yc = corner_coords(nx, ny, dx, p["dy"])
    b = np.minimum(-h_shelf, -h_off + np.maximum(Xc - x_toe, 0.0) * slope)
    yc = 0.5 * ny * p["dy"]
    r = np.hypot(Xc - island_x, Yc - yc)
    b = np.maximum(b, -h_shelf + island_h - np.maximum(r - island_r, 0.0) * island_slope)
    X, _ = cell_coords(nx, ny, dx, p["dy"])
    eta, P = solitary_profile(X, x0, rel_height * h_off, h_off)
    return dict(name=f"shelf_breaking_{nx}x{ny}", params=p, depth_c=-b, eta=eta, P=P, Q=np.zeros_like(eta),
                center=(island_x, yc), shore_radius=island_r + (island_h - h_shelf) / island_slope)


def rip_beach_scaled(nx, ny, seed=190904153, **kw):
    """rip_beach geometry scaled to an nx x ny grid covering the same 1024 m
    cross-shore extent (for parity tests at small sizes)."""
    dx = 1024.0 / nx
    return rip_beach(nx=nx, ny=ny, dx=dx, seed=seed, **kw)


# ---------------------------------------------------------------------------
# C4: 64 seeded domains of uneven size; C5: Poisson request stream
# ---------------------------------------------------------------------------

def beach_of_size(nx, ny, dx=0.1, rng=None, **kw):
    """C2-type domain scaled to nx x ny: offshore flat on the first 10 %, then
    a 1:20 beach crossing the still-water line 10 m further."""
    L = nx * dx
    return sloping_beach(nx=nx, ny=ny, dx=dx, x_toe=0.1 * L, **kw)


def solitary_of_size(nx, ny, dx=0.05, rng=None, **kw):
    """C1-type domain scaled to nx x ny (flat 1 m bed, 0.1 m solitary wave)."""
    x0 = 0.2 * nx * dx if rng is None else float(rng.uniform(0.15, 0.35)) * nx * dx
    return solitary_flat(nx=nx, ny=ny, dx=dx, x0=x0, steps=None, **kw)


def batch_mix(n=64, seed=190904154, nx_choices=None, ny_choices=None):
    rng = np.random.default_rng(seed)
    nx_choices = nx_choices if nx_choices is not None else list(range(256, 1537, 128))
    ny_choices = ny_choices if ny_choices is not None else list(range(256, 513, 64))
    out = []
    for k in range(n):
        nx = int(rng.choice(nx_choices))
        ny = int(rng.choice(ny_choices))
        if rng.uniform() < 0.5:
            s = solitary_of_size(nx, ny, rng=rng)
        else:
            s = beach_of_size(nx, ny, rng=rng)
        s["name"] = f"batch{k}_{s['name']}"
        out.append(s)
    return out


def request_work(spec):
    """Rough cell-steps of a request: cells x (t_end / Delta t), Delta t from
    the CFL number and the offshore long-wave speed."""
    p = spec["params"]
    h = float(np.max(spec["depth_c"]))
    dt = p["cfl"] * min(p["dx"], p["dy"]) / math.sqrt(G * h)
    return p["nx"] * p["ny"] * p["t_end"] / dt


def request_stream(n=200, seed=190904155, rho=0.8, capacity_cells_per_s=2.0e10, sides=None,
                   sim_seconds=(60.0, 600.0)):
    """Poisson arrivals of scenario requests of mixed size; returns a list of
    (arrival_time_s, spec) sorted by arrival.  Square sides log-uniform on
    [128, 2048] (multiples of 64), simulated durations uniform on
    sim_seconds, half plane beaches under a sine wavemaker (CFL 0.2), half
    rip-channel beaches under JONSWAP waves (2D: CFL 0.125, linear F*
    extrapolation), each with a seed of its own.  The arrival rate is set so
    that the offered load (request_work per second) is rho times the stated
    capacity in cell-steps per second."""
    rng = np.random.default_rng(seed)
    if sides is None:
        lo, hi = math.log(128), math.log(2048)
        sides = [int(round(math.exp(rng.uniform(lo, hi)) / 64.0)) * 64 for _ in range(n)]
    reqs = []
    work = []
    for k in range(n):
        side = max(128, min(2048, sides[k]))
        dur = float(rng.uniform(*sim_seconds))
        if rng.uniform() < 0.5:
            s = beach_of_size(side, side, dx=0.1, t_end=dur)
        else:
            s = rip_beach_scaled(side, side, seed=int(rng.integers(1 << 30)), t_end=dur, cfl=0.125,
                                 fstar_order=1)
        s["params"]["t_end"] = dur
        s["name"] = f"req{k}_{s['name']}"
        reqs.append(s)
        work.append(request_work(s))
    lam = rho * capacity_cells_per_s / float(np.mean(work))
    t = 0.0
    out = []
    for s in reqs:
        t += float(rng.exponential(1.0 / lam))
        out.append((t, s))
    return out


# ---------------------------------------------------------------------------
# small cases used by the physics pins and parity tests
# ---------------------------------------------------------------------------

def smooth_bump_bed(nx, ny, dx, depth=1.0, amp=0.3, seed=7, n_bumps=4):
    """Seeded smooth uneven bed, everywhere submerged (depth - bumps > 0)."""
    rng = np.random.default_rng(seed)
    Xc, Yc = corner_coords(nx, ny, dx, dx)
    Lx, Ly = nx * dx, ny * dx
    b = np.full_like(Xc, -depth)
    for _ in range(n_bumps):
        x0, y0 = rng.uniform(0.2, 0.8) * Lx, rng.uniform(0.2, 0.8) * Ly
        s = rng.uniform(0.08, 0.2) * min(Lx, Ly)
        b += rng.uniform(0.3, 1.0) * amp * np.exp(-((Xc - x0) ** 2 + (Yc - y0) ** 2) / (2 * s * s))
    return -b


def lake_at_rest(nx=48, ny=40, dx=0.1, seed=7, **kw):
    p = base_params(nx, ny, dx, **kw)
    depth_c = smooth_bump_bed(nx, ny, dx, seed=seed)
    eta, P, Q = rest_state(nx, ny)
    return dict(name="lake_at_rest", params=p, depth_c=depth_c, eta=eta, P=P, Q=Q)


def closed_basin_hump(nx=64, ny=48, dx=0.1, seed=11, amp=0.05, **kw):
    """Walls on all sides, uneven submerged bed, a Gaussian hump of water."""
    p = base_params(nx, ny, dx, **kw)
    depth_c = smooth_bump_bed(nx, ny, dx, seed=seed, amp=0.2)
    X, Y = cell_coords(nx, ny, dx, dx)
    rng = np.random.default_rng(seed)
    x0, y0 = rng.uniform(0.3, 0.7) * nx * dx, rng.uniform(0.3, 0.7) * ny * dx
    s = 0.1 * min(nx, ny) * dx
    eta = amp * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2 * s * s))
    return dict(name="closed_basin_hump", params=p, depth_c=depth_c, eta=eta, P=np.zeros_like(eta),
                Q=np.zeros_like(eta))


def standing_wave_1d(kd, cells_per_wavelength=64, depth=1.0, rel_amp=1e-4, ny=4, n_wavelengths=1, **kw):
    """Closed 1D basin holding n_wavelengths of a cos standing wave
    (eta = a cos(k x), P = Q = 0), walls on all sides, flat bed."""
    L = 2.0 * math.pi / (kd / depth) * n_wavelengths
    nx = cells_per_wavelength * n_wavelengths
    dx = L / nx
    p = base_params(nx, ny, dx, **kw)
    depth_c = np.full((ny + 1, nx + 1), float(depth))
    X, _ = cell_coords(nx, ny, dx, dx)
    k = kd / depth
    eta = rel_amp * depth * np.cos(k * X)
    return dict(name=f"standing_kd{kd}", params=p, depth_c=depth_c, eta=eta, P=np.zeros_like(eta),
                Q=np.zeros_like(eta), k=k, L=L)


def dam_break_dry_bed(nx=400, ny=4, dx=0.05, h_left=1.0, x_dam=None, **kw):
    """Ritter dam break: water of depth h_left for x < x_dam over a dry,
    horizontal bed lying at the still-water level, so d = 0 everywhere
    (the NLSW limit of the equations, Sec. 2)."""
    p = base_params(nx, ny, dx, **kw)
    depth_c = np.zeros((ny + 1, nx + 1))
    X, _ = cell_coords(nx, ny, dx, dx)
    x_dam = x_dam if x_dam is not None else 0.5 * nx * dx
    eta = np.where(X < x_dam, h_left, 0.0)
    return dict(name="dam_break", params=p, depth_c=depth_c, eta=eta, P=np.zeros_like(eta),
                Q=np.zeros_like(eta), x_dam=x_dam, h_left=h_left)
