#!/usr/bin/env python3
"""MACH-HOOI benchmark on one MI355X; prints one JSON line.

One step is the whole hot path over one synthetic window already resident
in HBM: the coin toss (with the sparse layouts), HOSVD initialisation,
`--sweeps` HOOI sweeps and the core.  The headline workload is the
monitoring-shaped hosts x metrics x minutes tensor 128 x 16 x 16384
(float32, Tucker rank (8,4,16) + diurnal sinusoids + Pareto spikes) at
p = 0.1, rank (8,4,16), 20 sweeps; the `voxel` block runs the 4-way
64 x 64 x 64 x 256 workload (p = 0.05, rank 10^4, 10 sweeps) the same way.

value = kept entries x sweeps / step time (sampled nnz per second of HOOI
sweeping, with sampling, HOSVD and core time included in the step).

roofline: the slower sparse tensor-times-matrix pass, timed per launch with
HIP events on its stream, cold (1 GiB written before each timed sweep, so
the kept entries come from HBM); warm figures beside.  Algorithmic bytes
per launch: 8 per kept entry (uint32 index + float32 value) plus the
float32 output and the segment pointers.

cpu_baseline: the FP64 numpy oracle on the benchmarked window, whole job
timed; accuracy: the device result of that window against the oracle's
(principal-angle sines, reconstruction errors e and e', core, fit).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

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
    ap.add_argument("--no-voxel", action="store_true",
                    help="skip the 64x64x64x256 voxel workload block")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="windows of the serving run after 100 warm-up windows (0: skip it)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times (the "
                         "reference kernel for scaling HBM counters; larger than the 256 MB "
                         "last-level cache, so that it streams from HBM)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the TTM traffic summary from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of this script with --copy-mib, and exit")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="write the kernel-time summary (profiles/) from a rocprofv3 --kernel-trace "
                         "--stats run of this script, and exit")
    ap.add_argument("--pmc-mfma", metavar="DIR",
                    help="write the MFMA utilisation summary of the Gram kernels from a rocprofv3 "
                         "--pmc run (SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE "
                         "SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_INSTS_VALU_MFMA_MOPS_BF16 "
                         "SQ_INSTS_VALU_MFMA_MOPS_F64) of this script, and exit")
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
            mt = re.search(r"k_rows_tiled<(\d+), (\d)>", n)
            key = None
            if m and m.group(5) == "0":      # float32 factors (the timed path)
                key = "ttm_tail_cols" if m.group(4) == "1" else "ttm_head_rows"
            elif mt and mt.group(2) == "0":
                key = "ttm_head_rows_tiles"
            elif "k_rows_tiled_sum" in n:
                key = "ttm_head_rows_sum"
            elif "copyBuffer" in n and int(r["Grid_Size"]) == big:
                key = "copy"
            if key:
                acc.setdefault(key, []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    fetch, write = read(fetch_dir, "FETCH_SIZE"), read(write_dir, "WRITE_SIZE")
    # the tiled head-row pass is two launches: tiles, then the partial sums
    for d in (fetch, write):
        if "ttm_head_rows_tiles" in d:
            d["ttm_head_rows"] = d.pop("ttm_head_rows_tiles") + d.pop("ttm_head_rows_sum", 0.0)
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
               "cd /tmp && export TMPDIR=/tmp && timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE "
               f"--output-format csv -d $R/{fd} -o run -- python3 $R/bench.py --steps 1 "
               f"--warmup 1 --no-cpu-baseline --serve-requests 0 --copy-mib {copy_mib}",
               f"(the same with --pmc WRITE_SIZE and -d $R/{wd})",
               f"python3 bench.py --pmc-summary {fd} {wd} --copy-mib {copy_mib}"]}
    return out


MFMA_JSON = os.path.join(ROOT, "profiles", "mfma_util_gram_kernels.json")


def source_digest(name):
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_0909_4969_amd", "csrc", name), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def mfma_summary(d):
    """Per-kernel MFMA figures of the Gram (and eigensolve) kernels from a
    counter CSV: utilisation = SQ_VALU_MFMA_BUSY_CYCLES (summed over SIMDs) /
    (device busy cycles x SIMDs), and the MFMA flops counted by
    SQ_INSTS_VALU_MFMA_MOPS_* (units of 512 flops), averaged over the
    dispatches of each kernel."""
    import csv
    import glob
    import re
    path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
    per = {}
    for r in csv.DictReader(open(path)):
        n = r["Kernel_Name"]
        m = re.search(r"(k_gram_y_mfma<\d+, \d>|k_gram_mfma<\d+, \w+>|k_mode_ss<\d+>|"
                      r"k_mode_solve<\d+, \d+>)", n)
        if not m:
            continue
        key = (m.group(1), r.get("Dispatch_Id", r.get("Correlation_Id", "")))
        per.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    acc = {}
    for (k, _), c in per.items():
        acc.setdefault(k, []).append(c)
    # GRBM_GUI_ACTIVE arrives summed over the XCDs: busy cycles of the
    # device = that sum / XCDs; SQ_VALU_MFMA_BUSY_CYCLES is summed over SIMDs.
    agent = [r for r in csv.DictReader(open(glob.glob(os.path.join(d, "**", "*agent_info.csv"),
                                                       recursive=True)[0])) if r["Agent_Type"] == "GPU"][0]
    nxcc, simds = int(agent["Num_Xcc"]), int(agent["Simd_Count"])
    out = {}
    for k, lst in sorted(acc.items()):
        def avg(name):
            return sum(x.get(name, 0.0) for x in lst) / len(lst)
        busy, gui = avg("SQ_VALU_MFMA_BUSY_CYCLES"), avg("GRBM_GUI_ACTIVE") / nxcc
        flops = 512.0 * (avg("SQ_INSTS_VALU_MFMA_MOPS_F32") + avg("SQ_INSTS_VALU_MFMA_MOPS_BF16") +
                         avg("SQ_INSTS_VALU_MFMA_MOPS_F64"))
        out[k] = {"dispatches": len(lst), "mfma_busy_cycles": busy, "gui_active_cycles": gui,
                  "mfma_util": round(busy / (gui * simds), 5) if gui else None,
                  "mfma_flops_per_dispatch": flops}
    rd = os.path.relpath(d, ROOT)
    return {"gram_source_digest": source_digest("gram.hip"), "kernels": out,
            "commands": ["cd /tmp && export TMPDIR=/tmp && timeout -s KILL 300 rocprofv3 --pmc "
                         "SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE SQ_INSTS_VALU_MFMA_MOPS_F32 "
                         "SQ_INSTS_VALU_MFMA_MOPS_BF16 SQ_INSTS_VALU_MFMA_MOPS_F64 --output-format csv "
                         f"-d $R/{rd} -o run -- python3 $R/bench.py --steps 1 --warmup 1 --no-cpu-baseline "
                         "--serve-requests 0",
                         f"python3 bench.py --pmc-mfma {rd}"]}


TRACE_MD = os.path.join(ROOT, "profiles", "kernels_monitoring-128x16x16384_voxel-64x64x64x256.md")


def trace_summary(d):
    """Markdown summary of a kernel trace of this script: the top kernels by
    total time, and the sparse passes split into cold launches (the first
    one after each 1 GiB cache flush) and warm ones."""
    import csv
    import glob
    import re
    rows = list(csv.DictReader(open(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)[0])))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))

    def short(n):
        n = n.replace("mach::(anonymous namespace)::", "").replace("mach::", "")
        return re.sub(r"\(.*$", "", n)
    tot = {}
    for r in rows:
        k = short(r["Kernel_Name"])
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        t = tot.setdefault(k, [0, 0.0, 1e30])
        t[0] += 1
        t[1] += dt
        t[2] = min(t[2], dt)
    # cold / warm split of the sparse passes (float32 variants); the tiled
    # head-row pass is its tile kernel plus the partial sum that follows
    passes = {"ttm_head_rows": [], "ttm_tail_cols": [], "voxel_head_rows": [], "voxel_tail_cols": []}
    flushed = False
    for i, r in enumerate(rows):
        n = r["Kernel_Name"]
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        if "FillFunctor<float>" in n and int(r["Grid_Size_X"]) >= (1 << 26):
            flushed = True
            continue
        key = None
        if "k_rows_tiled<16, 0>" in n:
            nxt = rows[i + 1] if i + 1 < len(rows) else None
            if nxt is not None and "k_rows_tiled_sum" in nxt["Kernel_Name"]:
                dt = (int(nxt["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            key = "ttm_head_rows"
        elif "k_spc<2, 8, 4, 1, 0, 1>" in n:
            key = "ttm_tail_cols"
        elif "k_spc<2, 16, 12, 0, 0, 0>" in n:
            key = "voxel_head_rows"
        elif "k_spc<2, 16, 12, 1, 0, 1>" in n:
            key = "voxel_tail_cols"
        if key:
            passes[key].append((flushed, dt))
            if key.endswith("tail_cols"):
                flushed = False
    total = sum(v[1] for v in tot.values())
    rd = os.path.relpath(d, ROOT)
    lines = ["# Kernel time of the benchmark run (monitoring window 128 x 16 x 16384 and voxel "
             "workload 64 x 64 x 64 x 256)", "",
             "Command (on the MI355X machine, repository root as `$R`):", "",
             "    cd /tmp && export TMPDIR=/tmp && timeout -k 10 300 rocprofv3 --kernel-trace --stats \\",
             f"      --output-format csv -d $R/{rd} -o run -- \\",
             "      python3 $R/bench.py --steps 2 --warmup 1 --no-cpu-baseline --serve-requests 0",
             f"    python3 bench.py --trace-summary {rd}", "",
             "Sparse passes (float32; the tiled head-row pass is its tile kernel through the end of its "
             "partial-sum kernel). Cold = the first pass of its kind after a 1 GiB buffer write "
             "(the cache flush of the bench's cold timing); warm = every other launch.", "",
             "| pass | cold launches | cold avg us | warm launches | warm avg us |", "|---|---:|---:|---:|---:|"]
    for k, v in passes.items():
        c = [dt for f, dt in v if f]
        w = [dt for f, dt in v if not f]
        if v:
            lines.append(f"| {k} | {len(c)} | {sum(c) / max(1, len(c)):.2f} | {len(w)} | "
                         f"{sum(w) / max(1, len(w)):.2f} |")
    lines += ["", f"Top kernels by total time (all kernels: {total / 1e3:.2f} ms):", "",
              "| kernel | calls | total ms | avg us | min us |", "|---|---:|---:|---:|---:|"]
    for k, (n, t, mn) in sorted(tot.items(), key=lambda kv: -kv[1][1])[:30]:
        lines.append(f"| {k} | {n} | {t / 1e3:.3f} | {t / n:.2f} | {mn:.2f} |")
    return "\n".join(lines) + "\n"


def mfma_from_profiles():
    """The committed MFMA summary if it was taken on the current Gram source."""
    try:
        with open(MFMA_JSON) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("gram_source_digest") != source_digest("gram.hip"):
        return None
    return {k: {"mfma_util": v["mfma_util"], "mfma_flops_per_dispatch": v["mfma_flops_per_dispatch"]}
            for k, v in d["kernels"].items() if k.startswith("k_gram")}


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


def cpu_baseline(X, p, seed, ranks, sweeps, nnz, runs):
    """The FP64 numpy oracle on the benchmarked window (window 0): coin toss,
    HOSVD, all sweeps and the core, timed in full on the host cores; then
    the device results of the same window (one per sweep precision)
    measured against it."""
    from threadpoolctl import threadpool_info

    from oracle import mach as O
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [os.cpu_count() or 1])
    t0 = time.perf_counter()
    Xh = O.sampled_tensor(X, p, seed, 0)
    t1 = time.perf_counter()
    A = O.hosvd_factors(Xh, ranks)
    t2 = time.perf_counter()
    fits = []
    n2 = float(np.sum(Xh * Xh))
    for _ in range(sweeps):
        A, tr = O.hooi_sweep(Xh, A, ranks)
        fits.append(O.fit_from_norms(n2, tr[-1]))
    t3 = time.perf_counter()
    G = O.core(Xh, A)
    t4 = time.perf_counter()
    t_job = t4 - t0
    del Xh
    cb = {
        "value": nnz * sweeps / t_job,
        "unit": "nnz/s",
        "cores": int(threads),
        "kind": "oracle",
        "cpu": cpu_model(),
        "sample": (f"FP64 numpy oracle on the benchmarked {'x'.join(map(str, X.shape))} window, whole job "
                   f"timed: coin toss {t1 - t0:.1f}s, HOSVD {t2 - t1:.1f}s, {sweeps} sweeps "
                   f"{t3 - t2:.1f}s, core {t4 - t3:.2f}s; job {t_job:.1f}s"),
    }
    e_o, e2_o = host_measures(X, G, A)
    acc = {"window": 0, "reference": "FP64 oracle, same coins, HOSVD + same sweeps + core",
           "oracle": {"rel_error_e": e_o, "rel_error_e_prime": e2_o, "fit": fits[-1]}}
    for name, r in runs.items():
        e_g, e2_g = host_measures(X, r["core"], r["factors"])
        acc[name] = {
            "sin_theta_per_mode": [float(f"{sin_theta_host(a, b):.3e}") for a, b in zip(A, r["factors"])],
            "rel_error_e": e_g, "e_over_oracle": e_g / e_o,
            "rel_error_e_prime": e2_g,
            "core_rel_diff": float(np.linalg.norm(r["core"] - G) / np.linalg.norm(G)),
            "fit": r["fit"],
        }
    acc["note"] = ("e = ||X - G x_n A_n|| / ||X|| (1 - the paper's accuracy); e' = ||X - X x_n A_n A_n^T|| "
                   "/ ||X||; sin theta = sine of the largest principal angle between the subspaces")
    return cb, acc


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


def serving_bench(n_requests, prec_modes, warmup_windows=100, saturated_windows=400):
    """Config-5 serving: Poisson arrivals (200/s) of hosts x 16 x T windows
    from 8 streams (hosts in {32, 64, 128} per stream, T uniform in
    [1024, 16384]), p = 0.05, ranks (8, 4, 16); a stream's first window runs
    HOSVD + 6 sweeps, later windows the warm time-mode update + 3 sweeps.
    Continuous batching (8 windows in flight over 8 HIP streams) against
    plain per-request solves (one window at a time).  Latency figures skip
    the first `warmup_windows` windows.  The saturated run queues
    `saturated_windows` windows at once (the device is never idle), so its
    rate is the throughput each mode can sustain."""
    import numpy as np
    import torch

    import synth
    from paper_0909_4969_amd import mach as M
    from paper_0909_4969_amd.serve import Engine, ServeConfig, latency_summary
    reqs = synth.serving_stream(n_requests=n_requests + warmup_windows)
    wins = device_windows(reqs)
    torch.cuda.synchronize()
    out = {"workload": f"poisson-200/s {n_requests} windows after {warmup_windows} warm-up, 8 streams, "
                       f"hosts x 16 x T, T in [1024,16384], p=0.05, ranks (8,4,16)",
           "windows_resident_in_hbm": True}
    modes = [("continuous_f32", dict(max_active=8, hip_streams=8), M.MACH_F32),
             ("per_request_f32", dict(max_active=1, hip_streams=1), M.MACH_F32)]
    modes += [(f"continuous_{name}", dict(max_active=8, hip_streams=8), code) for name, code in prec_modes]

    def work(cfg, res):
        return sum(r.nnz * ((cfg.sweeps_warm + 1.0 / 3.0) if r.warm else cfg.sweeps_cold) for r in res)

    for name, kw, prec in modes:
        cfg = ServeConfig(ranks=(8, 4, 16), p=0.05, sweeps_cold=6, sweeps_warm=3, prec=prec,
                          hbm_budget=64 << 30, **kw)
        eng = Engine(cfg)
        eng.run(wins[:8], realtime=False)            # kernels, allocator
        eng.resident.clear()
        torch.cuda.synchronize()
        res = eng.run(wins, realtime=True)
        kept = [r for r in res if r.req_id >= warmup_windows]
        summ = latency_summary(kept)
        summ["nnz_per_s"] = work(cfg, kept) / summ["span_s"]
        summ["mean_fit"] = float(np.mean([r.fit for r in kept]))
        summ["warm_windows"] = sum(1 for r in kept if r.warm)
        # saturated: every window queued at time 0
        eng.resident.clear()
        torch.cuda.synchronize()
        sat = eng.run(wins[:saturated_windows], realtime=False)
        span = max(r.done_s for r in sat) - min(r.admit_s for r in sat)
        summ["saturated"] = {"windows": len(sat), "span_s": round(span, 4),
                             "windows_per_s": round(len(sat) / span, 1),
                             "nnz_per_s": round(work(cfg, sat) / span, 1)}
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
        del eng, res, sat
        torch.cuda.synchronize()
    out["note"] = ("continuous: up to 8 windows in flight on 8 HIP streams, each window's kernels on its "
                   "own stream; per_request: one window at a time; mixed modes as in `precision`")
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def flush_caches(buf):
    """Writes a 1 GiB device buffer: evicts the 256 MB last-level cache and
    the L2s, so that the next kernel reads its inputs from HBM."""
    buf.fill_(1.0)


def run_workload(M, torch, X, shape, ranks, p, sweeps, seed, steps, warmup, cold_sweeps=10):
    """One workload: `warmup` untimed steps, `steps` timed whole steps
    (coin toss + layouts, HOSVD, sweeps, core; each window's status read
    before the next), per-phase times over PHASE_WINDOWS further windows,
    and the sparse passes timed warm (inside the timed steps, one launch in
    TIMING_EVERY) and cold (one sweep after each flush of the caches)."""
    dec = M.Decomposition(shape, ranks, p)

    def step(win):
        dec.sample(X, seed, win)
        dec.hosvd()
        for _ in range(sweeps):
            dec.sweep()
        dec.core()
        st = dec.status()[0]
        if st != 0:
            raise SystemExit(f"device status {st} ({M.status_string(st)}) in window {win}")

    for w in range(warmup):
        step(w)
    torch.cuda.synchronize()
    M.timing_enable(TIMING_EVERY)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record()
    for k in range(steps):
        step(warmup + k)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = e0.elapsed_time(e1) / steps
    nnz = dec.status()[1]
    warm = {0: M.timing_read(0), 1: M.timing_read(1)}
    M.timing_enable(0)

    names = ("sample_ms", "hosvd_ms", "sweeps_ms", "core_ms")
    per = {k: [] for k in names}
    for wi in range(PHASE_WINDOWS):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        dec.sample(X, seed, 1000 + wi)
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
    if dec.status()[0] != 0:
        raise SystemExit("device status after the per-phase windows")
    phase = {k: sum(v) / len(v) for k, v in per.items()}
    phase_range = {k: [round(min(v), 3), round(max(v), 3)] for k, v in per.items()}
    phase["sweep_ms"] = phase["sweeps_ms"] / sweeps

    # Cold: every timed sweep follows a 1 GiB write, so its sparse passes
    # read the kept entries from HBM.
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    M.timing_enable(1)
    for _ in range(cold_sweeps):
        flush_caches(flush)
        dec.sweep()
    torch.cuda.synchronize()
    cold = {0: M.timing_read(0), 1: M.timing_read(1)}
    M.timing_enable(0)
    del flush
    if dec.status()[0] != 0:
        raise SystemExit("device status after the cold sweeps")
    return dec, {"ms_step": ms_step, "wall": wall, "nnz": nnz, "phase": phase,
                 "phase_range": phase_range, "warm": warm, "cold": cold, "per": per}


def pass_roofline(shape, ranks, nnz, h, r):
    """Roofline of the slower sparse pass, timed cold; warm beside it."""
    d = len(shape)
    MH = int(np.prod(shape[:h]))
    MT = int(np.prod(shape[h:]))
    KT = int(np.prod(ranks[h:]))
    KH = int(np.prod(ranks[:h]))
    alg = {0: nnz * 8 + MH * KT * 4 + (MH + 1) * 4, 1: nnz * 8 + MT * KH * 4 + (MT + 1) * 4}
    name = {0: "ttm_head_rows", 1: "ttm_tail_cols"}
    out = {}
    for w in (0, 1):
        ms_c, n_c = r["cold"][w]
        ms_w, n_w = r["warm"][w]
        if n_c == 0 or n_w == 0:
            raise SystemExit("a sparse pass was not timed")
        out[w] = {"cold_us": ms_c / n_c * 1e3, "warm_us": ms_w / n_w * 1e3, "n_cold": n_c, "n_warm": n_w,
                  "bytes": alg[w]}
    dom = max(out, key=lambda w: out[w]["cold_us"])
    o = out[dom]
    achieved = o["bytes"] / (o["cold_us"] * 1e-6) / 1e9
    del d
    return {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic_from_profiles(name[dom]),
        "kernel": name[dom], "timing": "cold (1 GiB written before each timed sweep)",
        "avg_launch_us": round(o["cold_us"], 2), "launches": o["n_cold"],
        "algorithmic_bytes_per_launch": int(o["bytes"]),
        "warm": {"avg_launch_us": round(o["warm_us"], 2),
                 "achieved_GBs": round(o["bytes"] / (o["warm_us"] * 1e-6) / 1e9, 1),
                 "launches": o["n_warm"], "sampled_1_in": TIMING_EVERY},
        "other_pass": {name[w]: {"cold_us": round(v["cold_us"], 2), "warm_us": round(v["warm_us"], 2),
                                 "cold_GBs": round(v["bytes"] / (v["cold_us"] * 1e-6) / 1e9, 1),
                                 "algorithmic_bytes_per_launch": int(v["bytes"])}
                       for w, v in out.items() if w != dom},
    }


def host_measures(X_np, G, factors):
    """e = ||X - G x_n A_n|| / ||X|| and e' = ||X - X x_n A_n A_n^T|| / ||X||
    for orthonormal float64 factors, in float64 on the host."""
    X = np.asarray(X_np, np.float64)
    nx2 = float(np.sum(X * X))
    P = X
    for n, A in enumerate(factors):
        P = np.moveaxis(np.tensordot(np.asarray(A, np.float64), P, axes=(0, n)), 0, n)
    e = math.sqrt(max(0.0, nx2 - 2.0 * float(np.sum(P * G)) + float(np.sum(G * G))) / nx2)
    e2 = math.sqrt(max(0.0, nx2 - float(np.sum(P * P))) / nx2)
    return e, e2


def sin_theta_host(A_ref, A):
    A_ref, A = np.asarray(A_ref, np.float64), np.asarray(A, np.float64)
    return float(np.linalg.norm(A - A_ref @ (A_ref.T @ A), 2))


def main():
    args = parse()
    if args.trace_summary:
        md = trace_summary(args.trace_summary)
        with open(TRACE_MD, "w") as f:
            f.write(md)
        print(md)
        return
    if args.pmc_mfma:
        d = mfma_summary(args.pmc_mfma)
        with open(MFMA_JSON, "w") as f:
            json.dump(d, f, indent=1)
        print(json.dumps(d))
        return
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
    dec, r = run_workload(M, torch, X, shape, ranks, p, sweeps, args.seed, args.steps, args.warmup)
    nnz = r["nnz"]
    h, _ = M.layout_info(shape)
    value = nnz * sweeps / (r["ms_step"] / 1e3)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "nnz/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "monitoring-128x16x16384-f32", "p": p, "ranks": list(ranks),
                   "sweeps": sweeps, "nnz": nnz,
                   "step": "coin toss + layouts + HOSVD + sweeps + core",
                   "eigensolve_dtype": "f64"},
        "wall_s_timed": round(r["wall"], 3),
        "phases_ms": {k: round(v, 3) for k, v in r["phase"].items()},
        "phases_ms_range": r["phase_range"],
        "phases_windows": PHASE_WINDOWS,
        "sweep_only_nnz_per_s": round(nnz / (r["phase"]["sweep_ms"] / 1e3), 1),
        "roofline": pass_roofline(shape, ranks, nnz, h, r),
        "mfma": mfma_from_profiles(),
    }
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
    # A window slid by `hop` ticks along its stream: the toss of the new
    # window from the previous window's sample against a fresh toss.
    hop = shape[2] // 8
    Xs = torch.cat([X, X[..., :hop]], dim=2)
    Xa, Xb = Xs[..., :shape[2]].contiguous(), Xs[..., hop:].contiguous()
    del Xs
    prev = M.sample(Xa, p, args.seed, 0, cap=dec.cap, tick0=100000)
    slid = M.SampleWorkspace(shape, dec.cap, torch.empty_like(dec.sw.buf))
    for kind in ("slide", "fresh"):
        ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev2[0].record()
        for i in range(10):
            M.sample(Xb, p, args.seed, 0, ws=slid, tick0=100000 + hop,
                     prev=prev if kind == "slide" else None)
        ev2[1].record()
        torch.cuda.synchronize()
        coin_ms[kind] = ev2[0].elapsed_time(ev2[1]) / 10
    if slid.status()[0] != 0:
        raise SystemExit("device status after the slide comparison")
    del prev, slid, Xa, Xb
    out["stream_coins"] = {"sample_ms_window_coins": round(coin_ms["window"], 4),
                           "sample_ms_tick_coins": round(coin_ms["ticks"], 4),
                           "input_GBs_tick_coins": round(X.numel() * 4 / (coin_ms["ticks"] / 1e3) / 1e9, 1),
                           "slide_hop_ticks": hop,
                           "sample_ms_slid_window": round(coin_ms["slide"], 4),
                           "sample_ms_same_window_fresh": round(coin_ms["fresh"], 4),
                           "note": "coin toss + compaction + layouts of the window; tick coins "
                                   "keyed on (seed, series, absolute tick); the slid window reuses the "
                                   "previous window's coins and kept values for the shared ticks"}
    # The benchmarked window once more (window 0: HOSVD + sweeps + core) in
    # each sweep precision, for the precision comparison and the accuracy
    # against the oracle in the CPU leg.
    runs = {}
    for name, code in (("f32", M.MACH_F32), ("bf16", M.MACH_BF16), ("fp8", M.MACH_FP8E4M3)):
        dec.sample(X, args.seed, 0)
        dec.hosvd()
        torch.cuda.synchronize()
        eb0, eb1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        eb0.record()
        for _ in range(sweeps):
            dec.sweep(prec=code)
        eb1.record()
        dec.core()
        if dec.status()[0] != 0:
            raise SystemExit(f"device status of the {name} window")
        runs[name] = {"sweep_ms": eb0.elapsed_time(eb1) / sweeps,
                      "factors": [a.cpu().numpy() for a in dec.factors],
                      "core": dec.G.cpu().numpy(), "fit": float(dec.fit.item())}
    out["precision"] = {
        "window": 0,
        **{k: {"sweep_ms": round(v["sweep_ms"], 4), "fit": v["fit"]} for k, v in runs.items()},
        "note": "f32: float32 factor entries and Gram inputs; bf16: factor entries of the sparse passes "
                "and Gram inputs in bfloat16; fp8: factor entries in bfloat16, Gram inputs in OCP e4m3 "
                "scaled per tile; float32 accumulation and float64 eigensolve in all three",
    }
    del dec
    torch.cuda.synchronize()

    if not args.no_voxel:
        out["voxel"] = voxel_bench(M, torch, synth, args)
    out["tucker2"] = tucker2_bench(M, torch, synth)
    if args.copy_mib > 0:
        a = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.serve_requests > 0:
        out["serving"] = serving_bench(args.serve_requests, [("bf16", M.MACH_BF16),
                                                             ("fp8", M.MACH_FP8E4M3)])
    if not args.no_cpu_baseline:
        cb, acc = cpu_baseline(X_np, p, args.seed, ranks, sweeps, nnz, runs)
        out["cpu_baseline"] = cb
        out["accuracy"] = acc
    print(json.dumps(out), flush=True)


def tucker2_bench(M, torch, synth, sweeps=10, steps=3):
    """Tucker2 on the paper's sensor layout: 54 sensors x 4 measurement types
    x 5385 ticks (float32, a Tucker part of rank (5, 2, 6) + 5 % noise), the
    time mode left uncompressed, p = 0.1, ranks (5, 2): coin toss, HOSVD,
    `sweeps` sweeps and the core per step, each window's status read."""
    import numpy as np
    shape, ranks, p, seed = (54, 4, 5385), (5, 2, 0), 0.1, 20266
    X_np, _ = synth.workload1(shape=shape, ranks=(5, 2, 6), seed=seed, rel_noise=0.05)
    X = torch.from_numpy(X_np.astype(np.float32)).cuda()
    dec = M.Decomposition(shape, ranks, p)

    def step(win):
        dec.sample(X, seed, win)
        dec.hosvd()
        for _ in range(sweeps):
            dec.sweep()
        dec.core()
        if dec.status()[0] != 0:
            raise SystemExit("device status of the Tucker2 window")
    step(0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        step(1 + k)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nnz = dec.status()[1]
    return {"workload": "sensor-54x4x5385-f32, time mode uncompressed", "p": p, "ranks": [5, 2, "I"],
            "sweeps": sweeps, "nnz": nnz, "ms_per_step": round(ms, 3),
            "value": round(nnz * sweeps / (ms / 1e3), 1), "unit": "nnz/s", "fit": float(dec.fit.item()),
            "core_shape": list(dec.G.shape)}


def voxel_bench(M, torch, synth, args):
    """The 4-way voxel workload 64x64x64x256 (float32, core 10^4 with a
    geometrically decaying spectrum + 1 % noise) at p = 0.05, rank
    (10,10,10,10), 10 sweeps: whole-step throughput, phases and the sparse
    passes' roofline, as for the monitoring window."""
    shape, ranks, p, sweeps, seed = (64, 64, 64, 256), (10, 10, 10, 10), 0.05, 10, 20263
    X_np, _ = synth.workload3(shape)
    X = torch.from_numpy(X_np).cuda()
    del X_np
    dec, r = run_workload(M, torch, X, shape, ranks, p, sweeps, seed, max(2, args.steps // 2), 1)
    h, _ = M.layout_info(shape)
    nnz = r["nnz"]
    out = {"workload": "voxel-64x64x64x256-f32", "p": p, "ranks": list(ranks), "sweeps": sweeps,
           "nnz": nnz, "value": round(nnz * sweeps / (r["ms_step"] / 1e3), 1), "unit": "nnz/s",
           "ms_per_step": round(r["ms_step"], 3),
           "phases_ms": {k: round(v, 3) for k, v in r["phase"].items()},
           "phases_ms_range": r["phase_range"],
           "sweep_only_nnz_per_s": round(nnz / (r["phase"]["sweep_ms"] / 1e3), 1),
           "roofline": pass_roofline(shape, ranks, nnz, h, r)}
    out["roofline"]["traffic"] = None
    del dec, X
    torch.cuda.synchronize()
    return out


if __name__ == "__main__":
    main()
