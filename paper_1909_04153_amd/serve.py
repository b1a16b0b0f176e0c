"""Continuous-batching request loop over the C ABI.

Requests (scenario runs of mixed grid size, each with its own end time) arrive
over time.  A request is admitted when a slot is free and its device
workspace (``bq_workspace_bytes``) fits in the remaining HBM budget; admitted
domains keep their state resident on the device and advance together as one
batch (one launch per kernel per step), each with its own adaptive Delta t.
The batch membership changes only between step chunks.  A domain whose time
reaches its ``t_end`` latches a done status on the device and stops
advancing, so its result does not depend on when the host notices; the host
polls every chunk with one status readback for the whole batch, reads the
results of the finished members, frees their workspaces and records the
time-to-solution (arrival -> result on the host).  Member changes keep the
batch's device tables in the library's static array (no device allocation
in the loop; the step graphs are re-captured at the next chunk).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import bq


@dataclass
class Request:
    rid: int
    spec: dict
    arrival: float                      # seconds after the server's start
    admitted: float | None = None
    finished: float | None = None
    steps: int = 0
    t_sim: float = 0.0
    status: int | None = None
    cells: int = 0
    result: dict | None = None


@dataclass
class ServeStats:
    requests: list = field(default_factory=list)
    wall: float = 0.0
    cell_steps: float = 0.0

    def latencies(self, skip_before: float = 0.0):
        """times to solution of the requests arriving at or after
        skip_before; an unfinished request counts with the time it had
        waited when the run stopped (a lower bound: censored)"""
        return np.array([(r.finished if r.finished is not None else self.wall) - r.arrival
                         for r in self.requests if r.arrival >= skip_before and r.arrival <= self.wall])

    def summary(self, skip_before: float = 0.0):
        lat = self.latencies(skip_before)
        counted = [r for r in self.requests if skip_before <= r.arrival <= self.wall]
        censored = int(sum(r.finished is None for r in counted))
        return {"requests": len(self.requests), "completed": int(sum(r.finished is not None for r in self.requests)),
                "counted": len(counted), "censored": censored,
                "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
                "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
                "p99_is_lower_bound": censored > 0,
                "cell_steps_per_s": self.cell_steps / self.wall if self.wall > 0 else None,
                "wall_s": self.wall}


class Server:
    """Admission by HBM footprint + continuous batching of resident domains."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64, precision: int = bq.FP32,
                 chunk_steps: int = 16, keep_results: bool = False, static_tables: bool = True):
        import torch

        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        self.max_slots = int(max_slots)
        self.precision = precision
        self.chunk = int(chunk_steps)
        self.keep = keep_results
        self.static = static_tables
        self.stream = torch.cuda.Stream()
        self.queue: list[Request] = []
        self.active: list[tuple[Request, bq.Domain]] = []
        self.used = 0
        self.batch = None
        self.peak_used = 0

    def _footprint(self, spec):
        return bq.workspace_bytes(spec["params"], self.precision)

    def _admit(self, now):
        changed = False
        while self.queue and len(self.active) < self.max_slots:
            r = self.queue[0]
            if r.arrival > now:
                break
            need = self._footprint(r.spec)
            if need > self.budget:
                raise ValueError(f"request {r.rid} needs {need} B, more than the whole budget")
            if self.used + need > self.budget:
                break                      # FIFO: wait for memory to free up
            self.queue.pop(0)
            d = bq.Domain(r.spec["params"], r.spec["depth_c"], precision=self.precision, stream=self.stream)
            d.set_state(r.spec["eta"], r.spec["P"], r.spec["Q"])
            d.set_graph_steps(0)
            self.used += need
            self.peak_used = max(self.peak_used, self.used)
            r.admitted = now
            r.cells = d.nx * d.ny
            self.active.append((r, d))
            changed = True
        return changed

    def _retire(self, now, stats):
        # one readback for every member's latched status
        status, steps, tsim = self.batch.status()
        keep = []
        changed = False
        for (r, d), st, n, t in zip(self.active, status, steps, tsim):
            if st != bq.OK:
                if self.keep:
                    r.result = {f: d.read(f) for f in ("eta", "P", "Q")}
                r.finished = time.perf_counter() - self._t0
                r.status = int(st)
                r.steps = int(n)
                r.t_sim = float(t)
                self.used -= self._footprint(r.spec)
                d.close()
                changed = True
            else:
                keep.append((r, d))
        self.active = keep
        if changed and self.torch.cuda.memory_reserved() > self.budget + (4 << 30):
            # workspaces of retired requests sit in torch's cache; hand them
            # back before the cache outgrows the budget
            self.torch.cuda.empty_cache()
        return changed

    def run(self, requests: list[Request], max_wall: float = 600.0, progress=None,
            progress_every: float = 30.0) -> ServeStats:
        """serve the requests until all are done or max_wall seconds have
        passed; progress(msg), if given, is called every progress_every s"""
        stats = ServeStats(requests=list(requests))
        self.queue = sorted(requests, key=lambda r: r.arrival)
        self._t0 = time.perf_counter()
        next_report = progress_every
        while self.queue or self.active:
            now = time.perf_counter() - self._t0
            if now > max_wall:
                break
            if progress and now >= next_report:
                done = sum(r.finished is not None for r in stats.requests)
                progress(f"serve t={now:.0f}s: {done} done, {len(self.active)} resident "
                         f"({self.used / 2**30:.1f} GiB), {len(self.queue)} queued or not yet arrived")
                next_report += progress_every
            changed = self._admit(now)
            if not self.active:
                # idle until the next arrival
                time.sleep(max(0.0, min(0.01, self.queue[0].arrival - now)))
                continue
            if changed or self.batch is None:
                doms = [d for _, d in self.active]
                if self.batch is None:
                    self.batch = bq.Batch(doms, stream=self.stream)
                    self.batch.set_graph_steps(self.chunk)
                    if self.static:
                        self.batch.set(doms, static=True)
                else:
                    self.batch.set(doms, static=self.static)
            self.batch.step(self.chunk)
            if self._retire(now, stats) and self.active:
                self.batch.set([d for _, d in self.active], static=self.static)
        stats.wall = time.perf_counter() - self._t0
        if self.active:
            _, steps, tsim = self.batch.status()
            for (r, _), n, t in zip(self.active, steps, tsim):
                r.steps, r.t_sim = int(n), float(t)
        stats.cell_steps = float(sum(r.cells * r.steps for r in stats.requests))
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        return stats
