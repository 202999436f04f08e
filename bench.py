#!/usr/bin/env python3
"""MACH-HOOI benchmark on one MI355X; prints one JSON line.

One step is the whole hot path over one synthetic window already resident
in HBM: the coin toss (with the sparse layouts), HOSVD initialisation,
`--sweeps` HOOI sweeps and the core.  The workload is the monitoring-shaped
hosts x metrics x minutes tensor 128 x 16 x 16384 (float32, Tucker rank
(8,4,16) + diurnal sinusoids + Pareto spikes) at p = 0.1, rank (8,4,16),
20 sweeps.

value = kept entries x sweeps / step time (sampled nnz per second of HOOI
sweeping, with sampling, HOSVD and core time included in the step).

roofline: the sparse tensor-times-matrix pass that takes the most time,
timed per dispatch with HIP events over the timed steps; its algorithmic
bytes per launch are 8 bytes per kept entry (uint32 index + float32 value)
plus its float32 output and its segment pointers.

cpu_baseline: the FP64 numpy oracle on the same tensor (coin toss, HOSVD
and core timed in full; two sweeps timed and the rest extrapolated).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sampled nnz/s per HOOI sweep + p50/p99 window latency, mixed-prec vs FP32"
HBM_PEAK_GBS = 8000.0
TIMING_EVERY = 10      # timed sparse passes: one in every 10 of each kind
PHASE_WINDOWS = 5      # extra windows for the per-phase averages


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--p", type=float, default=0.1)
    ap.add_argument("--sweeps", type=int, default=20)
    ap.add_argument("--seed", type=int, default=20262)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=2)
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="windows of the serving run (0: skip it)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times (the "
                         "reference kernel for scaling HBM counters; larger than the 256 MB "
                         "last-level cache, so that it streams from HBM)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the TTM traffic summary from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of this script with --copy-mib, and exit")
    return ap.parse_args()


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "ttm_traffic_monitoring-128x16x16384.json")


def pmc_summary(fetch_dir, write_dir, copy_mib):
    """Per-launch HBM bytes of the two sparse TTM passes from rocprofv3
    counter CSVs: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) averaged over
    the dispatches of each kernel, each scaled by (true bytes of the
    reference copy) / (what the same counter reads for that copy)."""
    import csv
    import glob
    import re

    def read(d, counter):
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        # the reference copy: the copy kernel dispatches of the largest grid
        big = max(int(r["Grid_Size"]) for r in rows if "copyBuffer" in r["Kernel_Name"])
        acc = {}
        for r in rows:
            n = r["Kernel_Name"]
            m = re.search(r"k_spc<(\d), (\d+), (\d+), (\d), (\d)(?:, \d)?>", n)
            key = None
            if m and m.group(5) == "0":      # float32 factors (the timed path)
                key = "ttm_tail_cols" if m.group(4) == "1" else "ttm_head_rows"
            elif "copyBuffer" in n and int(r["Grid_Size"]) == big:
                key = "copy"
            if key:
                acc.setdefault(key, []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    fetch, write = read(fetch_dir, "FETCH_SIZE"), read(write_dir, "WRITE_SIZE")
    # the counter runs' output folders, relative to the repository root ($R)
    fd, wd = os.path.relpath(fetch_dir, ROOT), os.path.relpath(write_dir, ROOT)
    true_bytes = copy_mib * (1 << 20)
    f_scale = true_bytes / (fetch["copy"] * 1024.0)
    w_scale = true_bytes / (write["copy"] * 1024.0)
    out = {"ttm_source_digest": kernel_source_digest(),
           "fetch_kib_per_dispatch": {k: round(v, 1) for k, v in fetch.items()},
           "write_kib_per_dispatch": {k: round(v, 1) for k, v in write.items()},
           "copy_reference_bytes": true_bytes,
           "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
           "bytes_per_launch": {k: int(fetch[k] * 1024 * f_scale + write[k] * 1024 * w_scale)
                                for k in ("ttm_head_rows", "ttm_tail_cols")},
           "commands": [
               "cd /tmp && export TMPDIR=/tmp && timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE "
               f"--output-format csv -d $R/{fd} -o run -- python3 $R/bench.py --steps 1 "
               f"--warmup 1 --no-cpu-baseline --serve-requests 0 --copy-mib {copy_mib}",
               f"(the same with --pmc WRITE_SIZE and -d $R/{wd})",
               f"python3 bench.py --pmc-summary {fd} {wd} --copy-mib {copy_mib}"]}
    return out


def kernel_source_digest():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_0909_4969_amd", "csrc", "ttm.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(which):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_JSON) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("ttm_source_digest") != kernel_source_digest():
        return None
    return d.get("bytes_per_launch", {}).get(which)


def cpu_baseline(X, p, seed, ranks, sweeps, cpu_sweeps, nnz):
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import mach as O
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [os.cpu_count() or 1])
    t0 = time.perf_counter()
    Xh = O.sampled_tensor(X, p, seed, 0)
    t1 = time.perf_counter()
    A = O.hosvd_factors(Xh, ranks)
    t2 = time.perf_counter()
    for _ in range(cpu_sweeps):
        A, _ = O.hooi_sweep(Xh, A, ranks)
    t3 = time.perf_counter()
    O.core(Xh, A)
    t4 = time.perf_counter()
    per_sweep = (t3 - t2) / cpu_sweeps
    t_job = (t1 - t0) + (t2 - t1) + sweeps * per_sweep + (t4 - t3)
    del np
    return {
        "value": nnz * sweeps / t_job,
        "unit": "nnz/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"FP64 numpy oracle on the same {X.shape[0]}x{X.shape[1]}x{X.shape[2]} window: coin "
                   f"toss {t1 - t0:.1f}s, HOSVD {t2 - t1:.1f}s and core {t4 - t3:.2f}s timed in full, "
                   f"{cpu_sweeps} of {sweeps} sweeps timed ({per_sweep:.3f}s each) and the rest "
                   f"extrapolated; job {t_job:.1f}s"),
    }


def device_windows(reqs, metrics=16, ranks=(8, 4, 16), rel_noise=0.01):
    """Serving windows built on the device (seeded torch generators): per
    stream a Gaussian core and host/metric factors, per window a Gaussian
    time factor; X = Tucker product + noise of sigma = rel_noise ||X|| /
    sqrt(N), float32.  Same recipe as the host generator of the tests, drawn
    on the GPU so that hundreds of windows are ready in HBM in a second."""
    import torch
    from paper_0909_4969_amd.serve import Window
    per_stream = {}
    out = []
    for r in reqs:
        if r.stream_id not in per_stream:
            g = torch.Generator(device="cuda").manual_seed(r.seed)
            core = torch.randn(ranks, generator=g, device="cuda")
            A_h = torch.randn(r.hosts, ranks[0], generator=g, device="cuda") / r.hosts ** 0.5
            A_m = torch.randn(metrics, ranks[1], generator=g, device="cuda") / metrics ** 0.5
            T2 = torch.einsum("abc,ha,mb->hmc", core, A_h, A_m).reshape(r.hosts * metrics, ranks[2])
            per_stream[r.stream_id] = T2.contiguous()
        g = torch.Generator(device="cuda").manual_seed(r.seed * 1000003 + r.window_id)
        A_t = torch.randn(r.T, ranks[2], generator=g, device="cuda") / r.T ** 0.5
        X = (per_stream[r.stream_id] @ A_t.t().contiguous()).reshape(r.hosts, metrics, r.T)
        sigma = rel_noise * float(X.norm()) / X.numel() ** 0.5
        X = X + sigma * torch.randn(X.shape, generator=g, device="cuda")
        out.append(Window(r.req_id, r.stream_id, r.window_id, r.arrival_s, X.contiguous(), r.seed))
    return out


def serving_bench(n_requests, prec_modes):
    """Config-5 serving: Poisson arrivals (200/s) of hosts x 16 x T windows
    from 8 streams (hosts in {32, 64, 128} per stream, T uniform in
    [1024, 16384]), p = 0.05, ranks (8, 4, 16); a stream's first window runs
    HOSVD + 6 sweeps, later windows the warm time-mode update + 3 sweeps.
    Continuous batching (8 windows in flight over 4 HIP streams) against
    plain per-request solves (one window at a time)."""
    import numpy as np
    import torch

    import synth
    from paper_0909_4969_amd import mach as M
    from paper_0909_4969_amd.serve import Engine, ServeConfig, latency_summary
    reqs = synth.serving_stream(n_requests=n_requests)
    wins = device_windows(reqs)
    torch.cuda.synchronize()
    out = {"workload": f"poisson-200/s {n_requests} windows, 8 streams, hosts x 16 x T, "
                       f"T in [1024,16384], p=0.05, ranks (8,4,16)",
           "windows_resident_in_hbm": True}
    modes = [("continuous_f32", dict(max_active=8, hip_streams=4), M.MACH_F32),
             ("per_request_f32", dict(max_active=1, hip_streams=1), M.MACH_F32)]
    modes += [(f"continuous_{name}", dict(max_active=8, hip_streams=4), code) for name, code in prec_modes]
    for name, kw, prec in modes:
        cfg = ServeConfig(ranks=(8, 4, 16), p=0.05, sweeps_cold=6, sweeps_warm=3, prec=prec,
                          hbm_budget=64 << 30, **kw)
        eng = Engine(cfg)
        eng.run(wins[:8], realtime=False)            # warm-up: kernels, allocator
        eng.resident.clear()
        torch.cuda.synchronize()
        res = eng.run(wins, realtime=True)
        summ = latency_summary(res)
        work = sum(r.nnz * ((cfg.sweeps_warm + 1.0 / 3.0) if r.warm else cfg.sweeps_cold) for r in res)
        summ["nnz_per_s"] = work / summ["span_s"]
        summ["mean_fit"] = float(np.mean([r.fit for r in res]))
        summ["warm_windows"] = sum(1 for r in res if r.warm)
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
        del eng, res
        torch.cuda.synchronize()
    return out


def main():
    args = parse()
    if args.pmc_summary:
        d = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.copy_mib or 256)
        with open(TRAFFIC_JSON, "w") as f:
            json.dump(d, f, indent=1)
        print(json.dumps(d))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; --gpus must be 1 "
                                   "(the multi-GPU sharding is a design, not built)"}))
        sys.exit(2)
    import torch

    import synth
    from paper_0909_4969_amd import mach as M

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    shape, ranks, p, sweeps = (128, 16, 16384), (8, 4, 16), args.p, args.sweeps
    X_np, _ = synth.workload2(shape)
    X = torch.from_numpy(X_np).cuda()
    dec = M.Decomposition(shape, ranks, p)

    def step(win):
        dec.sample(X, args.seed, win)
        dec.hosvd()
        for _ in range(sweeps):
            dec.sweep()
        dec.core()
        # Each window's device status is read before its factors are used
        # (mach_read_status waits for the window's work on the stream).
        st = dec.status()[0]
        if st != 0:
            raise SystemExit(f"device status {st} ({M.status_string(st)}) in window {win}")

    for w in range(args.warmup):
        step(w)
    torch.cuda.synchronize()
    st, nnz, _ = dec.status()
    if st != 0:
        raise SystemExit(f"device status {st} ({M.status_string(st)}) after warmup")

    # Timed region: K whole steps, kernel timing of the sparse passes on (one
    # launch in every TIMING_EVERY of each kind, so that the event markers do
    # not weigh on the step time).
    M.timing_enable(TIMING_EVERY)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record()
    for k in range(args.steps):
        step(args.warmup + k)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    st, nnz, _ = dec.status()
    if st != 0:
        raise SystemExit(f"device status {st} ({M.status_string(st)})")
    rows_ms, rows_n = M.timing_read(0)
    cols_ms, cols_n = M.timing_read(1)
    M.timing_enable(0)

    # Per-phase times, averaged over PHASE_WINDOWS extra windows (not part of
    # the timed region; the sweep time varies from window to window).
    names = ("sample_ms", "hosvd_ms", "sweeps_ms", "core_ms")
    per = {k: [] for k in names}
    for wi in range(PHASE_WINDOWS):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        dec.sample(X, args.seed, 1000 + wi)
        ev[1].record()
        dec.hosvd()
        ev[2].record()
        for _ in range(sweeps):
            dec.sweep()
        ev[3].record()
        dec.core()
        ev[4].record()
        torch.cuda.synchronize()
        for i, k in enumerate(names):
            per[k].append(ev[i].elapsed_time(ev[i + 1]))
    phase = {k: sum(v) / len(v) for k, v in per.items()}
    phase_range = {k: [round(min(v), 3), round(max(v), 3)] for k, v in per.items()}
    phase["sweep_ms"] = phase["sweeps_ms"] / sweeps
    # The coin toss + layouts with stream (tick-keyed) coins against window
    # coins on the same window, 10 calls each (not part of the timed region).
    coin_ms = {}
    for kind in ("window", "ticks"):
        ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev2[0].record()
        for i in range(10):
            if kind == "ticks":
                dec.sample(X, args.seed, 0, tick0=1_000_000 + 997 * i)
            else:
                dec.sample(X, args.seed, 1000 + i)
        ev2[1].record()
        torch.cuda.synchronize()
        coin_ms[kind] = ev2[0].elapsed_time(ev2[1]) / 10
    if dec.status()[0] != 0:
        raise SystemExit("device status after the coin comparison")
    nnz_w, KT, KH = dec.status()[1], ranks[2], ranks[0] * ranks[1]
    MH, MT = shape[0] * shape[1], shape[2]

    passes = {
        "ttm_head_rows": (rows_ms, rows_n, nnz * 8 + MH * KT * 4 + (MH + 1) * 4),
        "ttm_tail_cols": (cols_ms, cols_n, nnz * 8 + MT * KH * 4 + (MT + 1) * 4),
    }
    if min(v[1] for v in passes.values()) == 0:
        raise SystemExit("no sparse pass was timed")
    dom = max(passes, key=lambda k: passes[k][0] / passes[k][1])
    ms_k, n_k, bytes_k = passes[dom]
    avg_s = ms_k / n_k / 1e3
    achieved = bytes_k / avg_s / 1e9
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic_from_profiles(dom),
        "kernel": dom, "avg_launch_us": round(avg_s * 1e6, 2), "launches": n_k, "sampled_1_in": TIMING_EVERY,
        "algorithmic_bytes_per_launch": int(bytes_k),
        "other_pass": {k: {"avg_launch_us": round(v[0] / v[1] * 1e3, 2),
                           "achieved_GBs": round(v[2] / (v[0] / v[1] / 1e3) / 1e9, 1)}
                       for k, v in passes.items() if k != dom},
    }
    value = nnz * sweeps / (ms_step / 1e3)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "nnz/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "monitoring-128x16x16384-f32", "p": p, "ranks": list(ranks),
                   "sweeps": sweeps, "nnz": nnz,
                   "step": "coin toss + layouts + HOSVD + sweeps + core",
                   "eigensolve_dtype": "f64"},
        "wall_s_timed": round(wall, 3),
        "phases_ms": {k: round(v, 3) for k, v in phase.items()},
        "phases_ms_range": phase_range,
        "phases_windows": PHASE_WINDOWS,
        "stream_coins": {"sample_ms_window_coins": round(coin_ms["window"], 4),
                         "sample_ms_tick_coins": round(coin_ms["ticks"], 4),
                         "input_GBs_tick_coins": round(X.numel() * 4 / (coin_ms["ticks"] / 1e3) / 1e9, 1),
                         "note": "coin toss + compaction + layouts of the window; tick coins "
                                 "keyed on (seed, series, absolute tick)"},
        "sweep_only_nnz_per_s": round(nnz / (phase["sweep_ms"] / 1e3), 1),
        "roofline": roofline,
    }
    # Mixed precision on the same window: 20 sweeps after HOSVD with bfloat16
    # factor entries in the sparse TTM, against the float32 run of the last
    # per-phase window above.
    A32 = [a.clone() for a in dec.factors]
    fit32 = float(dec.fit.item())
    last_win = 1000 + PHASE_WINDOWS - 1
    dec.sample(X, args.seed, last_win)
    dec.hosvd()
    torch.cuda.synchronize()
    eb0, eb1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    eb0.record()
    for _ in range(sweeps):
        dec.sweep(prec=M.MACH_BF16)
    eb1.record()
    torch.cuda.synchronize()
    if dec.status()[0] != 0:
        raise SystemExit("device status after the bfloat16 sweeps")
    import numpy as np
    sin_max = 0.0
    for a32, abf in zip(A32, dec.factors):
        a32, abf = a32.cpu().numpy(), abf.cpu().numpy()
        sin_max = max(sin_max, float(np.linalg.norm(abf - a32 @ (a32.T @ abf), 2)))
    out["precision"] = {
        "window": last_win,
        "f32": {"sweep_ms": round(per["sweeps_ms"][-1] / sweeps, 4), "fit": fit32},
        "bf16": {"sweep_ms": round(eb0.elapsed_time(eb1) / sweeps, 4), "fit": float(dec.fit.item()),
                 "max_sin_theta_vs_f32": sin_max},
        "note": "bf16 = sparse-TTM factor entries rounded to bfloat16, float32 sums, float64 eigensolve",
    }
    if args.copy_mib > 0:
        a = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.serve_requests > 0:
        out["serving"] = serving_bench(args.serve_requests, [("bf16", M.MACH_BF16)])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X_np, p, args.seed, ranks, sweeps, args.cpu_sweeps, nnz)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
