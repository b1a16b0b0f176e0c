"""Fixed versus adaptive time steps on the GPU (Sec. 5.1 Fig. 5.4, Sec. 5.2
Fig. 5.6-5.7, Sec. 5.4 Fig. 5.18).

The paper's claim: with the CFL-driven adaptive Delta t (Eq. 22, 47) a run
stays stable while taking far fewer steps than the largest fixed Delta t that
survives the same run, because the step only shrinks while the flow is fast
(a solitary wave running up an island) and recovers afterwards.  This module
measures that on a scenario: the adaptive Delta t trace, local CFL maps
(Eq. 22 per cell) at chosen times, the run-up record, and a bisection for the
largest stable fixed Delta t.  Every step runs in the HIP library; the host
only reads diagnostics back.

A run counts as stable when it reaches t_end with a finite state whose
local CFL number (Eq. 22 with the step taken) never exceeds `cfl_limit`
(1 by default: beyond it no explicit step of this scheme is stable, and a
growing instability passes it well before it overflows).  Energy is not a
usable criterion in run-up cases: the kinetic term (P^2 + Q^2) / 2h of thin
films at the wet/dry front grows without any instability.

    python -m paper_1909_04153_amd.robustness [--nx 601] [--t-end 20] [--fp64]
        [--scenario conical|shelf|rip] [--corrector] [--cfl C]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import bq
from . import scenarios as S


def run(spec, t_end, precision=bq.FP32, fixed_dt=None, every=1, snapshots=(), cfl_limit=1.0,
        max_steps=2_000_000):
    """Advance one domain to t_end; returns the Delta t trace (t, dt) every
    `every` steps, local-CFL statistics at the snapshot times and stability."""
    params = dict(spec["params"], t_end=float(t_end))
    if fixed_dt is not None:
        params.update(fixed_dt=1, dt_init=float(fixed_dt))
    d = bq.Domain(params, spec["depth_c"], precision=precision)
    d.set_state(spec["eta"], spec["P"], spec["Q"])
    d.set_graph_steps(0 if every < 16 else 16)
    i0 = d.sync()
    trace, snaps = [(i0.t, 0.0)], []
    cfl_seen = 0.0
    pending = sorted(float(s) for s in snapshots)
    stable, reason = True, "reached t_end"
    info = i0
    while True:
        d.step(every)
        info = d.sync()
        trace.append((info.t, info.dt_last))
        while pending and info.t >= pending[0]:
            c = d.read("cfl")
            snaps.append(dict(t=info.t, cfl_max=float(np.nanmax(c)), cfl_p99=float(np.nanpercentile(c, 99)),
                              cfl_mean=float(np.nanmean(c))))
            pending.pop(0)
        if info.status == bq.EDONE:
            break
        if info.status != bq.OK:
            stable, reason = False, bq.STATUS_NAMES.get(info.status, str(info.status))
            break
        cfl_now = info.smax * info.dt_last
        cfl_seen = max(cfl_seen, cfl_now)
        if not math.isfinite(cfl_now) or cfl_now > cfl_limit:
            stable, reason = False, f"local CFL number {cfl_now:.3g} at t = {info.t:.3f}"
            break
        if info.n >= max_steps:
            stable, reason = False, "step limit"
            break
    out = dict(stable=stable, reason=reason, steps=int(info.n), t=float(info.t), trace=trace, snapshots=snaps,
               cfl_max=cfl_seen, domain=d)
    return out


def runup_radii(spec, record, n_dir=16):
    """Horizontal run-up on an island, scaled by the still-water shoreline
    radius: for each of n_dir sectors (sector k spans the angles
    [2 pi k / n_dir, 2 pi (k+1) / n_dir) from the +x axis), the smallest
    distance from the island centre of a cell above still water that was
    inundated (finite run-up record), over the shoreline radius; 1 where no
    land cell of the sector was inundated."""
    nx, ny = spec["params"]["nx"], spec["params"]["ny"]
    dx, dy = spec["params"]["dx"], spec["params"]["dy"]
    X, Y = S.cell_coords(nx, ny, dx, dy)
    xc, yc = spec["center"]
    dc = spec["depth_c"]
    dcell = 0.25 * (dc[:-1, :-1] + dc[1:, :-1] + dc[:-1, 1:] + dc[1:, 1:])
    r = np.hypot(X - xc, Y - yc)
    ang = np.mod(np.arctan2(Y - yc, X - xc), 2.0 * math.pi)
    hit = np.isfinite(record) & (dcell < 0.0)
    out = []
    for k in range(n_dir):
        lo, hi = 2.0 * math.pi * k / n_dir, 2.0 * math.pi * (k + 1) / n_dir
        m = hit & (ang >= lo) & (ang < hi)
        out.append(float(r[m].min() / spec["shore_radius"]) if m.any() else 1.0)
    return out


def largest_stable_fixed_dt(spec, t_end, lo, hi, precision=bq.FP32, rel_tol=0.03, every=64, log=None):
    """Geometric bisection between a stable `lo` and an unstable `hi`."""
    runs = []

    def one(dt):
        r = run(spec, t_end, precision, fixed_dt=dt, every=every)
        r["domain"].close()
        runs.append((dt, r["stable"], r["steps"], r["reason"]))
        if log:
            log(f"fixed dt {dt:.6g}: {'stable' if r['stable'] else 'unstable'} after {r['steps']} steps "
                f"({r['reason']})")
        return r["stable"]

    if not one(lo):
        return None, runs
    if one(hi):
        return hi, runs
    while hi / lo > 1.0 + rel_tol:
        mid = math.sqrt(lo * hi)
        if one(mid):
            lo = mid
        else:
            hi = mid
    return lo, runs


def study(nx=601, t_end=20.0, precision=bq.FP32, snapshots=(4.0, 7.0, 10.0, 14.0), log=None, corrector=False,
          cfl=None, scenario="conical"):
    """The fixed-versus-adaptive comparison on the conical-island basin (Sec.
    5.1) at nx x nx cells over the same 30 m, or (scenario "shelf") on the
    breaking solitary wave over a shelf with an island (Sec. 5.2) at
    nx x nx/5 cells over the same 40 m x 8 m, or (scenario "rip") on the rip
    beach under irregular (JONSWAP) waves from rest (Sec. 5.4) at nx x nx
    cells over 1024 m; optionally with the Adams-Moulton corrector and
    another CFL target."""
    kw = {}
    if corrector:
        kw.update(corrector=1, fstar_order=2)
    if cfl is not None:
        kw.update(cfl=float(cfl))
    if scenario == "shelf":
        spec = S.shelf_breaking(nx=nx, ny=nx // 5, dx=40.0 / nx, **kw)
    elif scenario == "rip":
        kw.setdefault("cfl", 0.125)
        kw.setdefault("fstar_order", 1)
        spec = S.rip_beach_scaled(nx, nx, **kw)
    else:
        dx = 30.0 / (nx - 1) if nx != 601 else 0.05
        spec = S.conical_island(nx=nx, ny=nx, dx=dx, **kw)
    t0 = time.perf_counter()
    ad = run(spec, t_end, precision, snapshots=snapshots)
    t_ad = time.perf_counter() - t0
    if log:
        log(f"adaptive: {'stable' if ad['stable'] else 'unstable'} after {ad['steps']} steps to t = {ad['t']:.3f}")
    dts = np.array([dt for _, dt in ad["trace"][1:]])
    # run-up around an island (the rip beach has none)
    radii = runup_radii(spec, ad["domain"].read("runup")) if "center" in spec else None
    ad["domain"].close()
    lo, hi = 0.1 * float(dts.min()), 4.0 * float(dts.max())
    t0 = time.perf_counter()
    best, runs = largest_stable_fixed_dt(spec, t_end, lo, hi, precision, log=log)
    t_fx = time.perf_counter() - t0
    res = dict(
        scenario=spec["name"], t_end=t_end, precision="fp32" if precision == bq.FP32 else "fp64",
        corrector=bool(corrector), cfl=spec["params"]["cfl"], fstar_order=spec["params"]["fstar_order"],
        adaptive=dict(stable=ad["stable"], reason=ad["reason"], steps=ad["steps"], dt_first=float(dts[0]),
                      dt_min=float(dts.min()), dt_max=float(dts.max()), dt_mean=float(ad["t"] / ad["steps"]),
                      t_min_dt=float(ad["trace"][1 + int(np.argmin(dts))][0]), seconds=t_ad,
                      cfl_max=ad["cfl_max"],
                      cfl_snapshots=ad["snapshots"], runup_over_shoreline_radius=radii),
        fixed=dict(largest_stable_dt=best, steps_at_that_dt=(int(math.ceil(t_end / best)) if best else None),
                   runs=[dict(dt=a, stable=b, steps=c, reason=d) for a, b, c, d in runs], seconds=t_fx),
    )
    if best:
        res["steps_fixed_over_adaptive"] = res["fixed"]["steps_at_that_dt"] / ad["steps"]
    # a coarse trace (every ~1 % of the run) for plots
    tr = ad["trace"]
    stride = max(1, len(tr) // 100)
    res["adaptive"]["trace"] = [(float(t), float(dt)) for t, dt in tr[1::stride]]
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--nx", type=int, default=601)
    ap.add_argument("--t-end", type=float, default=20.0)
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--corrector", action="store_true", help="AB3 predictor + Adams-Moulton corrector")
    ap.add_argument("--cfl", type=float, default=None, help="CFL target of the adaptive run")
    ap.add_argument("--scenario", choices=("conical", "shelf", "rip"), default="conical")
    ap.add_argument("--snapshots", default="4,7,10,14", help="times of the local CFL maps, comma separated")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    res = study(a.nx, a.t_end, bq.FP64 if a.fp64 else bq.FP32, log=lambda m: print(m, flush=True),
                corrector=a.corrector, cfl=a.cfl, scenario=a.scenario,
                snapshots=tuple(float(v) for v in a.snapshots.split(",") if v))
    txt = json.dumps(res)
    print(txt, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")


if __name__ == "__main__":
    main()
