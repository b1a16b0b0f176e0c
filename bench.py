#!/usr/bin/env python
"""Throughput benchmark of the HIP time step on one MI355X.

Default workload: 64 seeded domains of uneven size (256..1536 x 256..512
cells, C1-type solitary waves on a flat bed and C2-type sloping beaches under
a sine wavemaker) advanced together in FP32, one launch per kernel per step,
steps replayed from hipGraphs.  A step is one time step of every domain:
Delta t from the CFL maximum, fluxes, dispersion, friction, AB3 update, both
tridiagonal line solves, boundary ghosts.

Prints one JSON line: Gcell-steps/s (interior cells x steps / s), the HBM
roofline of the dominant kernel (algorithmic bytes / its mean duration, HIP
events on the launch stream), the single-domain FP64 rates, the error of
each FP32 line against the FP64 path after the same steps, and the CPU
oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "Gcell-steps/s + % HBM peak (FP32 batched vs FP64 plain); p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per interior cell and step, per kernel (field words x
# word size): the stencil/update kernel reads w, P^{n,n-1,n-2}, Q^{n,n-1,n-2},
# the bed and E/F/G^{n-1,n-2} (14 words) and writes E/F/G^n, w^{n+1} and the
# two line-solve right-hand sides (6 words); the finalize kernel reads the two
# right-hand sides and writes P^{n+1}, Q^{n+1} (4 words); 24 words in all.
WORDS = {"k_dt": 0, "k_rhs": 20, "k_reduced": 0, "k_final": 4}
WORDS_STEP = 24
# measured HBM traffic (PMC FETCH_SIZE / WRITE_SIZE, scaled by a plain copy's
# reading) is kept with the profile summaries, tagged with a hash of the
# kernel sources it was taken on; it is reported only while they match
PROFILE_SUMMARIES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ("paper_1909_04153_amd/csrc/bq_kernels.hpp", "paper_1909_04153_amd/csrc/bq_layout.hpp",
                  "paper_1909_04153_amd/csrc/bq_lib.hip")


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_record(tag, kernel, workload_name, dtype, lanes):
    """the `tag:` record of the committed counter summaries for this kernel,
    workload, lane count and the current kernel sources, or None"""
    want = kernel_source_hash()
    if not os.path.isdir(PROFILE_SUMMARIES):
        return None
    for fn in sorted(os.listdir(PROFILE_SUMMARIES)):
        with open(os.path.join(PROFILE_SUMMARIES, fn)) as fh:
            for line in fh:
                if not line.startswith(tag + ":"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                if (kv.get("kernel") == kernel and kv.get("workload") == workload_name
                        and kv.get("dtype") == dtype and kv.get("lanes", "1") == str(lanes)
                        and kv.get("source_sha256_16") == want):
                    return kv
    return None


def measured_traffic(kernel, workload_name, dtype, lanes):
    """HBM bytes per launch (FETCH_SIZE / WRITE_SIZE, calibrated) from the
    committed counter summaries, or None"""
    kv = _profile_record("traffic", kernel, workload_name, dtype, lanes)
    return float(kv["bytes_per_launch"]) if kv else None


SIMDS, CLOCK_HZ, CYCLES_PER_VALU = 1024, 2.4e9, 4   # MI355X: 256 CUs x 4 SIMDs; wave64 FP32 op in 4 cycles


def valu_issue(kernel, workload_name, dtype, mean_ms):
    """VALU issue time of one launch (SQ_INSTS_VALU / SQ_WAVES from the
    committed counter summaries x waves x 4 cycles over 1024 SIMDs at
    2.4 GHz) against its measured duration, or None"""
    kv = _profile_record("valu", kernel, workload_name, dtype, 1)
    if not kv or not mean_ms:
        return None
    ipw, waves = float(kv["insts_per_wave"]), float(kv["waves_per_launch"])
    issue_ms = ipw * waves * CYCLES_PER_VALU / (SIMDS * CLOCK_HZ) * 1e3
    return {"insts_per_wave": ipw, "waves_per_launch": waves, "issue_ms": issue_ms,
            "frac": issue_ms / mean_ms}


def workload(name):
    from paper_1909_04153_amd import scenarios as S

    if name == "batch64":
        return S.batch_mix(64, seed=190904154), "fp32"
    if name == "beach1024x256":
        return [S.sloping_beach()], "fp32"
    if name == "beach1024x256_fp64":
        return [S.sloping_beach()], "fp64"
    if name == "rip2048":
        return [S.rip_beach(cfl=0.125, fstar_order=1)], "fp32"
    if name == "solitary200x20":
        return [S.solitary_flat()], "fp64"
    raise SystemExit(f"unknown workload {name}")


def make_group(bq, specs, dtype, lanes=2, batch=False):
    """the domains and what advances them: the domain itself, or a batch
    (always for several domains; for one domain when `batch`, so that its
    schedule can be tuned)"""
    prec = bq.FP32 if dtype == "fp32" else bq.FP64
    doms = [bq.domain_from_spec(s, precision=prec) for s in specs]
    if len(doms) == 1 and not batch:
        return doms, doms[0]
    return doms, bq.Batch(doms, lanes=lanes)


def tuned(group, args):
    """apply the autotuned (or cached) schedule to a batch; returns it"""
    if args.no_autotune or not hasattr(group, "autotune"):
        return None
    t = group.autotune(steps_per_trial=32, cache=args.tune_cache)
    return {k: t[k] for k in ("lanes", "graph_steps", "reduce_block", "reduce_segments", "swizzle", "cached")}


def timed(torch, group, steps, warmup):
    group.step(warmup)
    group.wait()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    group.step(steps)
    group.wait()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def single_line(bq, torch, args, wl, steps):
    """one domain (as a batch of one, schedule tuned): throughput, and the
    simulated seconds advanced per wall-clock second over the timed steps"""
    sp, dt_ = workload(wl)
    ds, g = make_group(bq, sp, dt_, batch=True)
    sched = tuned(g, args)
    c = sum(s_["params"]["nx"] * s_["params"]["ny"] for s_ in sp)
    g.step(args.warmup)
    g.wait()
    t_a = ds[0].sync().t
    e = timed(torch, g, steps, 0)
    t_b = ds[0].sync().t
    wsize = 4 if dt_ == "fp32" else 8
    out = {"value": c * steps / e / 1e9, "unit": "Gcell-steps/s", "ms_per_step": e / steps * 1e3, "cells": c,
           "steps": steps, "schedule": sched, "sim_s_per_wall_s": (t_b - t_a) / e,
           "effective_hbm_frac": WORDS_STEP * wsize * c * steps / e / 1e9 / HBM_PEAK_GBS}
    del g, ds
    torch.cuda.synchronize()
    if dt_ == "fp32":
        out["fp32_error"] = fp32_error(bq, torch, sp, steps)
    return out


def fp32_error(bq, torch, specs, steps):
    """Error of the FP32 path stated against the FP64 path (whose parity with
    the FP64 oracle, relative L2 <= 1e-12 per step, the GPU tests hold): both
    advance the same initial states `steps` adaptive steps; per domain
    ||eta32 - eta64|| / ||eta64||, worst and median over the domains."""
    etas = {}
    for dt_ in ("fp32", "fp64"):
        ds, g = make_group(bq, specs, dt_, lanes=1)
        g.step(steps)
        g.wait()
        etas[dt_] = [d.read("eta") for d in ds]
        if g is not ds[0]:
            g.close()
        for d in ds:
            d.close()
        del g, ds
        torch.cuda.synchronize()
    errs = [float(np.linalg.norm(a - b) / max(float(np.linalg.norm(b)), 1e-300))
            for a, b in zip(etas["fp32"], etas["fp64"])]
    return {"reference": "fp64 path", "steps": steps, "domains": len(errs),
            "eta_rel_l2_max": max(errs), "eta_rel_l2_median": float(np.median(errs))}


def cpu_baseline(specs, budget_s):
    """the oracle as it stands, one host core, on a bounded sample"""
    from oracle.oracle import OracleDomain

    done_cells = 0
    used = 0.0
    names = []
    for s in specs:
        o = OracleDomain(s["params"], s["depth_c"])
        o.set_state(s["eta"], s["P"], s["Q"])
        n = s["params"]["nx"] * s["params"]["ny"]
        steps = 0
        t0 = time.perf_counter()
        while True:
            rc = o.step(1)
            steps += 1
            el = time.perf_counter() - t0
            if rc != 0 or el > budget_s / 4 or used + el > budget_s:
                break
        used += el
        done_cells += n * steps
        names.append(f"{s['name']} x {steps} steps")
        o.close()
        if used >= budget_s:
            break
    return done_cells / used, used, names


def _oracle_worker(args):
    spec, budget_s = args
    from oracle.oracle import OracleDomain

    o = OracleDomain(spec["params"], spec["depth_c"])
    o.set_state(spec["eta"], spec["P"], spec["Q"])
    n = spec["params"]["nx"] * spec["params"]["ny"]
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        if o.step(1) != 0:
            break
        steps += 1
    el = time.perf_counter() - t0
    o.close()
    return n * steps, el


def cpu_baseline_all_cores(specs, budget_s, cores):
    """one oracle process per core on distinct domains of the batch (the
    oracle itself is single-threaded): aggregate cell-steps/s"""
    import multiprocessing as mp

    jobs = [(specs[k % len(specs)], budget_s) for k in range(cores)]
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs)
    return sum(c / e for c, e in res if e > 0)


def copy_bandwidth(torch, bq=None, mib=1024, reps=5):
    """device-to-device copy of `mib` MiB, (read + write) bytes / time: the
    library's hand-written copy kernel (16 bytes per lane) when `bq` is
    given, else torch's copy"""
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.ones(n, dtype=torch.uint8, device="cuda")

    def copy():
        if bq is not None:
            bq.stream_copy(a, b)
        else:
            a.copy_(b)

    copy()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        copy()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n / (ms * 1e-3) / 1e9


def fp32_error_run(bq, torch, spec, t_end, checkpoints=4):
    """FP32 against FP64 over a whole run: both paths advance the same
    initial state to t_end (each with its own adaptive Delta t); eta relative
    L2 and largest pointwise difference over the wave amplitude at
    `checkpoints` evenly spaced times (the nearest step at or after each)"""
    amp = max(float(np.max(np.abs(spec["eta"]))), float(np.sum(np.abs(spec["params"].get("wave_amp", [])))))
    marks = [t_end * (k + 1) / checkpoints for k in range(checkpoints)]
    res = {}
    for dt_, prec in (("fp32", bq.FP32), ("fp64", bq.FP64)):
        d = bq.domain_from_spec(spec, precision=prec)
        d.set_graph_steps(16)
        snaps, steps = [], 0
        t0 = time.perf_counter()
        for tm in marks:
            while d.sync().t < tm:
                d.step(16)
            i = d.sync()
            assert i.status == bq.OK, (dt_, i)
            snaps.append((i.t, i.n, d.read("eta")))
        res[dt_] = (snaps, time.perf_counter() - t0)
        d.close()
        torch.cuda.synchronize()
    rows = []
    for (t32, n32, e32), (t64, n64, e64) in zip(res["fp32"][0], res["fp64"][0]):
        rows.append({"t32": t32, "t64": t64, "steps32": n32, "steps64": n64,
                     "eta_rel_l2": float(np.linalg.norm(e32 - e64) / max(float(np.linalg.norm(e64)), 1e-300)),
                     "eta_max_over_amp": float(np.max(np.abs(e32 - e64))) / amp})
    return {"reference": "fp64 path", "t_end": t_end, "checkpoints": rows,
            "wall_s": {"fp32": res["fp32"][1], "fp64": res["fp64"][1]}}


def serve_run(bq, seconds):
    """a reduced Poisson request stream (48 requests, sides 128..1024, 2..12 s
    simulated each) through the continuous-batching loop; the configured
    stream (200 requests, 128..2048, 60..600 s) runs with --serve-c5"""
    from paper_1909_04153_amd import scenarios as S
    from paper_1909_04153_amd import serve

    rng = np.random.default_rng(190904155)
    n = 48
    reqs = []
    t = 0.0
    for k in range(n):
        side = int(round(math.exp(rng.uniform(math.log(128), math.log(1024))) / 64.0)) * 64
        dur = float(rng.uniform(2.0, 12.0))
        if rng.uniform() < 0.5:
            spec = S.beach_of_size(side, side, dx=0.1, t_end=dur)
        else:
            spec = S.rip_beach_scaled(side, side, seed=int(rng.integers(1 << 30)), t_end=dur, cfl=0.125,
                                      fstar_order=1)
        spec["params"]["t_end"] = dur
        t += float(rng.exponential(seconds / n / 2.0))
        reqs.append(serve.Request(k, spec, arrival=t))
    budget = 16 << 30
    srv = serve.Server(budget, max_slots=32, precision=bq.FP32, chunk_steps=16)
    stats = srv.run(reqs, max_wall=4.0 * seconds)
    out = stats.summary(skip_before=0.1 * t)
    out["cell_steps_per_s"] = out["cell_steps_per_s"] / 1e9 if out["cell_steps_per_s"] else None
    out["unit_throughput"] = "Gcell-steps/s"
    out["stream"] = "reduced: 48 requests, sides 128..1024, 2..12 s simulated, first 10 % of arrivals excluded"
    out["hbm_budget_bytes"] = budget
    out["peak_resident_bytes"] = srv.peak_used
    return out


def serve_c5(bq, torch, rho, n_req=200, max_wall=1100.0, chunk=16, warmup_s=10.0, seed=190904155):
    """The configured serving stream: n_req Poisson arrivals of C2-type
    beaches and C3-type rip beaches, square sides log-uniform on
    [128, 2048], 60..600 s simulated each, offered load rho times the
    capacity (measured first: the cell-steps/s of a batch of 16 requests of
    the stream's own mix), HBM admission on a 200 GiB budget, up to 64
    resident; p50/p99 time to solution over the requests arriving after the
    first warmup_s seconds (unfinished ones count with the time they had
    waited: censored, and p99 is then a lower bound)."""
    from paper_1909_04153_amd import scenarios as S
    from paper_1909_04153_amd import serve

    t_gen = time.perf_counter()
    print(f"serving stream: generating {n_req} requests", file=sys.stderr, flush=True)
    probe = S.request_stream(n=n_req, seed=seed, rho=1.0, capacity_cells_per_s=1.0)
    # capacity: a batch of 16 requests of the mix, 200 steps (FP32, 2 lanes)
    sample = [s for _, s in probe[:16]]
    doms = [bq.domain_from_spec(s, precision=bq.FP32) for s in sample]
    b = bq.Batch(doms)
    b.set_graph_steps(chunk)
    b.step(32)
    b.sync()
    cells = sum(d.nx * d.ny for d in doms)
    t0 = time.perf_counter()
    b.step(200)
    b.sync()
    cap = cells * 200 / (time.perf_counter() - t0)
    print(f"serving stream: capacity {cap / 1e9:.1f} Gcell-steps/s on a batch of 16 requests", file=sys.stderr,
          flush=True)
    b.close()
    for d in doms:
        d.close()
    del doms, b, sample
    torch.cuda.synchronize()
    # the stream itself: the same requests, the interarrival times (drawn
    # for rho 1 at a capacity of 1 cell-step/s) scaled to rho at the
    # measured capacity
    stream = [(t / (rho * cap), sp) for t, sp in probe]
    del probe
    work = [S.request_work(s) for _, s in stream]
    reqs = [serve.Request(k, s, arrival=t) for k, (t, s) in enumerate(stream)]
    gen_s = time.perf_counter() - t_gen
    budget = 200 << 30
    srv = serve.Server(budget, max_slots=64, precision=bq.FP32, chunk_steps=chunk)
    stats = srv.run(reqs, max_wall=max_wall, progress=lambda m: print(m, file=sys.stderr, flush=True))
    out = stats.summary(skip_before=warmup_s)
    out["cell_steps_per_s"] = out["cell_steps_per_s"] / 1e9 if out["cell_steps_per_s"] else None
    span = stream[-1][0]
    out.update({"rho": rho, "unit_throughput": "Gcell-steps/s", "capacity_gcs": cap / 1e9,
                "arrival_span_s": span, "offered_gcs": sum(work) / span / 1e9,
                "estimated_work_gcs": sum(work) / 1e9,
                "warmup_excluded_s": warmup_s, "hbm_budget_bytes": budget, "max_slots": 64,
                "peak_resident_bytes": srv.peak_used, "chunk_steps": chunk, "generation_s": gen_s,
                "stream": f"{n_req} requests, sides 128..2048 log-uniform, 60..600 s simulated, "
                          "half beaches (CFL 0.2), half rip beaches (CFL 0.125), seed %d" % seed})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batch64")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--lanes", type=int, default=2, choices=(1, 2, 3, 4),
                    help="launch lanes of a batch (two groups on two streams, or one) with --no-autotune")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default batch schedule instead of running the library's autotuner")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of autotuned schedules per batch shape (read, and written after tuning)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="run the request loop for about this long and report p50/p99 (0 = skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (5 times), for counter calibration")
    ap.add_argument("--serve-c5", type=float, default=0.0, metavar="RHO",
                    help="only run the configured serving stream (200 requests, 128..2048, 60..600 s) at this "
                         "offered load and print its JSON line")
    ap.add_argument("--serve-max-wall", type=float, default=1100.0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "domains are independent, so a multi-GPU run is one such process per GPU", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20)
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.ones(n, dtype=torch.uint8, device="cuda")
        for _ in range(5):
            a.copy_(b)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "repeats": 5}))
        return

    from paper_1909_04153_amd import bq

    bq.load()
    if args.serve_c5 > 0:
        print(json.dumps({"metric": "p50/p99 time to solution", "serving_c5": serve_c5(
            bq, torch, args.serve_c5, max_wall=args.serve_max_wall)}), flush=True)
        return
    specs, dtype = workload(args.workload)
    cells = sum(s["params"]["nx"] * s["params"]["ny"] for s in specs)
    # a single-domain workload runs as a batch of one, so that its schedule
    # is tuned like the other lines'
    doms, group = make_group(bq, specs, dtype, args.lanes, batch=not args.no_autotune)
    schedule = None
    if isinstance(group, bq.Batch):
        if not args.no_autotune:
            # trial steps are ordinary steps of the batch, before the warm-up
            schedule = group.autotune(steps_per_trial=32, cache=args.tune_cache)
        schedule = dict(group.tune, **({"cached": schedule["cached"]} if schedule else {"autotuned": False}))
    lanes = getattr(group, "lanes", 1)
    el = timed(torch, group, args.steps, args.warmup)
    value = cells * args.steps / el / 1e9
    ms_step = el / args.steps * 1e3
    for d in doms:
        st = d.sync().status
        if st != 0:
            raise SystemExit(f"domain {d.params} latched status {st}")
    # Per-kernel durations with HIP events on the launch stream (plain
    # launches).  The roofline is taken with one lane, each kernel alone on
    # the GPU and one launch covering every cell; with several lanes the
    # kernels of the groups share the GPU, so their event times are also given.
    kms2 = None
    if lanes > 1:
        kms2 = group.profile(args.profile_steps)
        group.set_lanes(1)
    kms = group.profile(args.profile_steps)
    if lanes > 1:
        group.set_lanes(lanes)
    dom_k = max(kms, key=kms.get)
    wsize = 4 if dtype == "fp32" else 8
    cells_launch = cells
    achieved = WORDS[dom_k] * wsize * cells_launch / (kms[dom_k] * 1e-3) / 1e9 if WORDS[dom_k] else None
    roof = {"bound": "hbm", "kernel": dom_k, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": measured_traffic(dom_k, args.workload, dtype, 1), "traffic_unit": "bytes/launch",
            "algorithmic_bytes_per_cell": WORDS[dom_k] * wsize, "cells_per_launch": cells_launch,
            "mean_ms": kms[dom_k], "profiled": "one lane, plain launches, HIP events on the launch stream",
            "valu_issue": valu_issue(dom_k, args.workload, dtype, kms[dom_k])}
    out = {"metric": METRIC, "value": value, "unit": "Gcell-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": {"workload": args.workload, "domains": len(specs), "cells": cells,
                      "precision": dtype, "lanes": lanes, "schedule": schedule},
           "effective_hbm_frac": WORDS_STEP * wsize * cells * args.steps / el / 1e9 / HBM_PEAK_GBS,
           "kernels_ms": kms, "roofline": roof}
    if kms2 is not None:
        out["kernels_ms_lanes"] = kms2
    del group, doms
    torch.cuda.synchronize()
    if dtype == "fp32":
        out["fp32_error"] = fp32_error(bq, torch, specs, args.steps)
    out["copy_gbs"] = copy_bandwidth(torch)
    # the achievable HBM rate: the library's hand-written copy kernel
    out["copy_gbs_hip"] = copy_bandwidth(torch, bq)
    if achieved:
        roof["achievable_peak"] = out["copy_gbs_hip"]
        roof["frac_of_achievable"] = achieved / out["copy_gbs_hip"]
    out["effective_frac_of_achievable"] = out["effective_hbm_frac"] * HBM_PEAK_GBS / out["copy_gbs_hip"]
    tr = roof["traffic"]
    if tr:
        roof["traffic_gbs"] = tr / (kms[dom_k] * 1e-3) / 1e9
        roof["traffic_frac"] = roof["traffic_gbs"] / HBM_PEAK_GBS
    if not args.no_fp64:
        # single domains in FP32: C3 (2048 x 2048 rip beach) and C2 (1024 x
        # 256 beach)
        out["fp32_single_c3"] = single_line(bq, torch, args, "rip2048", max(20, args.steps // 2))
        out["fp32_single_c2"] = single_line(bq, torch, args, "beach1024x256", max(20, args.steps))
        # the same 64-domain batch with the Adams-Moulton corrector (two
        # passes of the stencil and the line solves per step)
        sp, dt_ = workload("batch64")
        for s_ in sp:
            s_["params"] = dict(s_["params"], corrector=1)
        ds, g = make_group(bq, sp, dt_, args.lanes)
        sched_pc = tuned(g, args)
        c = sum(s_["params"]["nx"] * s_["params"]["ny"] for s_ in sp)
        n = max(20, args.steps // 2)
        e = timed(torch, g, n, args.warmup)
        out["fp32_batch64_corrector"] = {"value": c * n / e / 1e9, "unit": "Gcell-steps/s",
                                         "ms_per_step": e / n * 1e3, "cells": c, "steps": n, "schedule": sched_pc}
        del g, ds
        torch.cuda.synchronize()
        fp64 = {}
        for wl in ("beach1024x256_fp64", "solitary200x20"):
            fp64[wl] = single_line(bq, torch, args, wl, max(20, args.steps))
        out["fp64_plain"] = fp64
        # FP32 against FP64 over whole runs: the 1024 x 256 beach over its
        # 20 s (wave through the wet/dry shoreline), and the 2048^2 rip beach
        # over 30 s from a state with the JONSWAP train already in the domain
        from paper_1909_04153_amd import scenarios as S

        out["fp32_error_runs"] = {
            "beach1024x256_20s": fp32_error_run(bq, torch, S.sloping_beach(), 20.0),
            "rip2048_spun_up_30s": fp32_error_run(
                bq, torch, S.spun_up(S.rip_beach(cfl=0.125, fstar_order=1), h_taper=(0.4, 0.25)), 30.0)}
    if args.serve_seconds > 0:
        out["serving"] = serve_run(bq, args.serve_seconds)
    if not args.no_cpu_baseline:
        rate, used, names = cpu_baseline(specs, args.cpu_seconds)
        out["cpu_baseline"] = {"value": rate / 1e9, "unit": "Gcell-steps/s", "cores": 1, "kind": "oracle",
                               "seconds": used, "sample": "; ".join(names),
                               "host_cpus": os.cpu_count()}
        cores = max(1, min(16, os.cpu_count() or 1))
        agg = cpu_baseline_all_cores(specs, args.cpu_seconds / 2, cores)
        out["cpu_baseline_all_cores"] = {"value": agg / 1e9, "unit": "Gcell-steps/s", "cores": cores,
                                         "kind": "oracle", "sample": f"{cores} processes, one batch domain each, "
                                                                     f"{args.cpu_seconds / 2:.0f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
