"""Serving loop for MACH-HOOI over tensor-stream windows.

Monitoring data arrives as windows (hosts x metrics x T) of several
streams (Section 1: a monitoring system decomposes each new window; Remark 2:
the coin is tossed as each measurement arrives, so a window can be sampled
as soon as it is complete).  The engine

  * admits arrived windows while the device memory they need (dense window,
    sample and solver workspaces, factors, core; all from the library's size
    queries) fits an HBM budget and an active-slot limit;
  * keeps several windows on the device at once, each on its own HIP stream,
    so their kernels overlap (continuous batching: a window joins as soon as
    a slot and memory free up and leaves as soon as its result is ready);
  * warm-starts a stream's next window from the host and metric factors of
    its previous window, which stay resident: the time mode is updated first
    from them (a sweep that starts at the last mode), then full HOOI sweeps
    run (Alg. 2); a stream's first window is initialised by HOSVD;
  * samples a window that carries its absolute first tick with stream coins,
    from the stream's previous window's sample when they overlap (the shared
    measurements keep their coins and kept values; only the new ticks are
    tossed and read);
  * reports each window's latency (result ready - arrival).

Argument marshalling and scheduling only: every step of a window runs in the
library's HIP kernels.  Windows of one stream are processed in arrival order
(the warm start needs the previous result); windows of different streams
overlap freely.  Results do not depend on what else is running: every window
has its own workspaces and the kernels are deterministic.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import torch

from . import mach as M


@dataclass
class Window:
    """One request: a device-resident float32 window of one stream.  With
    tick0 (the absolute tick of the window's first time step) the coins are
    keyed on (seed, series, tick), so windows of a stream that overlap in time
    keep the same measurements; else on (seed, window_id, position)."""
    req_id: int
    stream_id: int
    window_id: int
    arrival_s: float
    X: torch.Tensor
    seed: int
    tick0: int | None = None


@dataclass
class ServeConfig:
    ranks: tuple = (8, 4, 16)
    p: float = 0.05
    sweeps_cold: int = 6          # HOOI sweeps after HOSVD (first window of a stream)
    sweeps_warm: int = 3          # full sweeps after the warm time-mode update
    prec: int = M.MACH_F32
    hbm_budget: int = 32 << 30    # bytes the in-flight windows may hold
    max_active: int = 8           # windows on the device at once
    hip_streams: int = 4          # HIP streams the windows are spread over
    warm_start: bool = True


@dataclass
class WindowResult:
    req_id: int
    stream_id: int
    window_id: int
    warm: bool
    nnz: int
    fit: float
    factors: list
    core: torch.Tensor
    arrival_s: float
    admit_s: float
    done_s: float
    footprint: int

    @property
    def latency_ms(self) -> float:
        return 1e3 * (self.done_s - self.arrival_s)


@dataclass
class _Job:
    win: Window
    stream: torch.cuda.Stream
    warm: bool
    footprint: int
    admit_s: float
    sw: M.SampleWorkspace
    solver: torch.Tensor
    factors: list
    fit: torch.Tensor
    G: torch.Tensor
    norm2: torch.Tensor
    done: torch.cuda.Event = field(default=None)


class Engine:
    def __init__(self, cfg: ServeConfig, device="cuda"):
        self.cfg = cfg
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max(1, cfg.hip_streams))]
        self._load = [0] * len(self.streams)
        self.resident = {}        # stream_id -> (hosts, [A_host, A_metric]) float64 device tensors
        # stream_id -> the last window's sample workspace, kept when its
        # window carried an absolute tick: the stream's next window is
        # sampled from it (shared measurements keep their coins and values)
        self.prev_sample = {}

    # ---- memory ----------------------------------------------------------
    def footprint(self, shape) -> int:
        """Device bytes a window of this shape holds while in flight."""
        shape = tuple(int(x) for x in shape)
        cap = M.nnz_capacity(shape, self.cfg.p)
        b = 4 * int(torch.tensor(shape).prod())                      # the dense window
        b += M.sample_workspace_bytes(shape, cap)
        b += M.solver_workspace_bytes(shape, self.cfg.ranks, cap)
        b += sum(8 * I * R for I, R in zip(shape, self.cfg.ranks))   # factors
        b += 8 * int(torch.tensor(self.cfg.ranks).prod()) + 64       # core, fit, norm
        return b

    # ---- one window ------------------------------------------------------
    def _launch(self, win: Window, now_s: float) -> _Job:
        cfg = self.cfg
        shape = tuple(win.X.shape)
        si = min(range(len(self.streams)), key=lambda i: self._load[i])
        self._load[si] += 1
        s = self.streams[si]
        res = self.resident.get(win.stream_id)
        warm = cfg.warm_start and res is not None and res[0] == shape[0]
        with torch.cuda.stream(s):
            cap = M.nnz_capacity(shape, cfg.p)
            sw = M.SampleWorkspace(shape, cap, torch.empty(M.sample_workspace_bytes(shape, cap),
                                                           dtype=torch.uint8, device=self.device))
            solver = M.solver_workspace(shape, cfg.ranks, cap, self.device)
            fit = torch.zeros(1, dtype=torch.float64, device=self.device)
            G = torch.empty(tuple(cfg.ranks), dtype=torch.float64, device=self.device)
            norm2 = torch.empty(1, dtype=torch.float64, device=self.device)
            prev = self.prev_sample.get(win.stream_id) if win.tick0 is not None else None
            if prev is not None and (prev.shape != shape or prev.cap != cap):
                prev = None
            M.sample(win.X, cfg.p, win.seed, win.window_id, ws=sw, stream=s, tick0=win.tick0, prev=prev)
            if warm:
                factors = [res[1][0].clone(), res[1][1].clone(),
                           torch.zeros(shape[2], cfg.ranks[2], dtype=torch.float64, device=self.device)]
                M.solver_reset(shape, cfg.ranks, solver, stream=s)
                M.hooi_sweep(sw, cfg.ranks, factors, solver, first_mode=len(shape) - 1, fit=fit,
                             prec=cfg.prec, stream=s)
                sweeps = cfg.sweeps_warm
            else:
                factors = M.hosvd(sw, cfg.ranks, solver, stream=s)
                sweeps = cfg.sweeps_cold
            for _ in range(sweeps):
                M.hooi_sweep(sw, cfg.ranks, factors, solver, fit=fit, prec=cfg.prec, stream=s)
            M.core(sw, cfg.ranks, factors, solver, G, norm2, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        job = _Job(win, s, warm, self.footprint(shape), now_s, sw, solver, factors, fit, G, norm2, ev)
        job._si = si
        return job

    def _finish(self, job: _Job, now_s: float) -> WindowResult:
        st, nnz, _ = job.sw.status(job.solver, stream=job.stream)
        if st != M.MACH_OK:
            raise M.MachError(f"window {job.win.req_id}", st)
        self._load[job._si] -= 1
        w = job.win
        if self.cfg.warm_start:
            self.resident[w.stream_id] = (w.X.shape[0], [job.factors[0], job.factors[1]])
        if w.tick0 is not None:
            self.prev_sample[w.stream_id] = job.sw
        return WindowResult(w.req_id, w.stream_id, w.window_id, job.warm, nnz, float(job.fit.item()),
                            job.factors, job.G, w.arrival_s, job.admit_s, now_s, job.footprint)

    # ---- the loop --------------------------------------------------------
    def run(self, windows, realtime=True, poll_s=20e-6):
        """Serves `windows` (arrival_s relative to the start of the call).
        With realtime=False every window counts as arrived at time 0."""
        cfg = self.cfg
        todo = collections.deque(sorted(windows, key=lambda w: (w.arrival_s, w.req_id)))
        waiting = collections.deque()
        active = []
        results = []
        busy_streams = set()
        used = 0
        t0 = time.perf_counter()
        while todo or waiting or active:
            now = time.perf_counter() - t0
            while todo and (not realtime or todo[0].arrival_s <= now):
                waiting.append(todo.popleft())
            progressed = False
            # completions first: they free slots, memory and streams
            still = []
            for job in active:
                if job.done.query():
                    results.append(self._finish(job, time.perf_counter() - t0))
                    used -= job.footprint
                    busy_streams.discard(job.win.stream_id)
                    progressed = True
                else:
                    still.append(job)
            active = still
            # admission: arrival order, one window per data stream at a time
            held = set()
            keep = collections.deque()
            while waiting:
                w = waiting.popleft()
                if w.stream_id in busy_streams or w.stream_id in held:
                    held.add(w.stream_id)
                    keep.append(w)
                    continue
                fp = self.footprint(w.X.shape)
                if fp > cfg.hbm_budget:
                    raise M.MachError(f"window {w.req_id} needs {fp} bytes, over the HBM budget",
                                      M.MACH_ENOMEM)
                if len(active) < cfg.max_active and used + fp <= cfg.hbm_budget:
                    active.append(self._launch(w, time.perf_counter() - t0))
                    used += fp
                    busy_streams.add(w.stream_id)
                    progressed = True
                else:
                    held.add(w.stream_id)
                    keep.append(w)
            waiting = keep
            if not progressed:
                if active:
                    time.sleep(poll_s)
                elif todo:
                    time.sleep(max(0.0, min(todo[0].arrival_s - (time.perf_counter() - t0), 1e-3)))
        results.sort(key=lambda r: r.req_id)
        return results


def latency_summary(results):
    """p50 / p99 / max latency (ms) and aggregate sampled nnz per second of
    HOOI sweeping (sum of nnz x sweeps over the served span)."""
    import numpy as np
    lat = np.array([r.latency_ms for r in results])
    span = max(r.done_s for r in results) - min(r.arrival_s for r in results)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "windows": len(results), "span_s": span}
