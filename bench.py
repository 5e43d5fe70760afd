"""Benchmark: UMI window-estimates/s on one MI355X.

Workload: 1,000 TESS-sector light curves of 18,000 samples (2-min cadence),
W = 361, alpha = 2, c = 5, 5 iterations, each curve with a 1-day NaN gap in
the middle -- synthetic, seeded (synth.config_batch(1)).  One step is one
umi_detrend_batch call over the whole packed batch (segmentation pre-pass +
the persistent estimate kernel), with inputs already resident in HBM.

Prints ONE JSON line with the throughput, the main kernel's place on the
FP32 VALU roofline (timed live with HIP events on the launch stream), and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "window-estimates/s (1000x18k TESS batch, W=361); p50/p99 latency in serve loop"
PEAK_FP32_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0
TARGET_FRAC = 0.5          # the batched kernel's goal: half the FP32 VALU peak


# Algorithmic FP32 work per window sample (add/sub/mul = 1, fma = 2; compares,
# selects, the median and the per-window divides and square root not counted):
# Phase 2 costs 3 (subtract, fused square-accumulate); each Phase 3 iteration
# costs 8 (residual 1, scaling 1, 1 - u^2 2, square 1, two accumulations 1 + 2).


def window_sizes(batch, gap_days: float = 0.5) -> np.ndarray:
    """Samples n in each output's window (0 where the output is NaN), counted
    on the host from the input layout alone -- valid samples, segments broken
    at time steps above `gap_days`, segments shorter than W/3 dropped,
    windows cut at segment ends.  Used only to count algorithmic work."""
    out = np.zeros(batch.n_samples, np.int64)
    for b in range(batch.n_curves):
        f, t, W = batch.curve(b)
        o = int(batch.offsets[b])
        h = (W - 1) // 2
        valid = np.isfinite(f) & np.isfinite(t)
        idx = np.flatnonzero(valid)
        if idx.size == 0:
            continue
        breaks = np.flatnonzero(np.diff(t[idx]) > gap_days) + 1
        for seg in np.split(idx, breaks):
            if seg.size < max(1, W // 3):
                continue
            lo, hi = seg[0], seg[-1]
            csum = np.concatenate([[0], np.cumsum(valid[lo:hi + 1])])
            a = np.maximum(seg - h, lo) - lo
            e = np.minimum(seg + h, hi) - lo + 1
            out[o + seg] = csum[e] - csum[a]
    return out


def cpu_model() -> dict:
    """What the host says about its CPU (Linux): the model string, family /
    model / stepping, clock, and lscpu's view when it is there."""
    info = {"model_name": "unknown"}
    keys = {"model name": "model_name", "vendor_id": "vendor", "cpu family": "family",
            "model": "model", "stepping": "stepping", "cpu MHz": "mhz"}
    try:
        with open("/proc/cpuinfo") as fh:
            block = fh.read().split("\n\n")[0]  # the first processor
        for line in block.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys:
                info[keys[k.strip()]] = v.strip()
    except OSError:
        pass
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            k = k.strip()
            if k in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                     "CPU max MHz", "Hypervisor vendor"):
                info["lscpu_" + k.lower().replace(" ", "_").replace("(s)", "s")] = v.strip()
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(batch, budget_s: float = 15.0, first_curves: int | None = None,
                 total_windows: int | None = None):
    """The oracle as it stands, on the host's cores, over the first curves of
    the same workload: about `budget_s` seconds, or exactly `first_curves`
    curves.  With `total_windows` (the whole workload's finite outputs) the
    time the oracle would take for all of it is extrapolated at the measured
    rate."""
    import oracle
    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, int(cores))
    if first_curves is None:
        # one curve per thread, so the probe sees the parallel rate
        probe = min(int(batch.n_curves), max(8, cores))
        sub = batch_prefix(batch, probe)
        t0 = time.perf_counter()
        oracle.detrend_batch(sub.flux, sub.time, sub.lengths, sub.W, n_threads=cores)
        per_curve = (time.perf_counter() - t0) / probe
        n = int(min(batch.n_curves, max(probe, round(budget_s / max(per_curve, 1e-6)))))
    else:
        n = int(min(batch.n_curves, first_curves))
    sub = batch_prefix(batch, n)
    t0 = time.perf_counter()
    tr, _ = oracle.detrend_batch(sub.flux, sub.time, sub.lengths, sub.W, n_threads=cores)
    dt = time.perf_counter() - t0
    windows = int(np.isfinite(tr).sum())
    used = min(cores, n)  # the oracle runs one curve per thread
    out = {"value": windows / dt, "unit": "window-estimates/s", "cores": used,
           "kind": "oracle", "cpu": cpu_model(),
           "per_core": windows / dt / max(1, used),
           "sample": "first %d of the %d curves (%d windows), FP64 C oracle, %d threads, %.1f s"
                     % (n, batch.n_curves, windows, used, dt)}
    if total_windows is not None:
        out["extrapolated_full_workload_s"] = total_windows / (windows / dt)
        out["extrapolation"] = ("all %d windows of the workload at the sampled rate (curves of "
                                "this workload are drawn independently, so the first ones are a "
                                "fair sample of its length and W mix)" % total_windows)
    return out


WORKLOADS = {0: "tess_single_20k_w361", 1: "tess_batch_1000x18k_w361",
             2: "kepler_ragged_2000x40k-70k_w25", 3: "mixed_ragged_10000x1k-120k_wmix"}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2604_06602_amd", "csrc", f)
                  for f in ("umi_kernels.hip", "umi_internal.h")]


def counted_traffic(workload):
    """HBM bytes per main-kernel launch on `workload` from the committed
    counter summary, or None when there is none or the kernel sources changed
    after those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "umi_main_kernel__%s.md" % WORKLOADS[workload])
    try:
        text = open(path).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(("kernel_source_sha256:", "hbm_traffic_bytes_per_launch:")))
    if fields.get("kernel_source_sha256", "").strip() != h.hexdigest():
        return None
    try:
        return int(fields["hbm_traffic_bytes_per_launch"].strip())
    except (KeyError, ValueError):
        return None


def measured_fma_peak(torch, stream, log, iters=40000, launches=10):
    """Sustained scalar FP32 FMA rate of this GPU (TFLOP/s): the measurement
    aid in libumi_diag.so (16 independent FMA chains per thread, 8 waves per
    SIMD, packed forms disabled as for the library), timed with HIP events on
    `stream`."""
    import ctypes
    path = os.path.join(ROOT, "paper_2604_06602_amd", "libumi_diag.so")
    lib = ctypes.CDLL(path)
    lib.umi_diag_fma_peak.restype = ctypes.c_int32
    lib.umi_diag_fma_peak.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    grid = cus * 8  # 8 workgroups of 4 waves per CU: 8 waves per SIMD
    out = torch.empty(grid * 256, dtype=torch.float32, device="cuda")
    flop = ctypes.c_double()
    h = ctypes.c_void_p(int(stream.cuda_stream))

    def launch():
        st = lib.umi_diag_fma_peak(iters, grid, ctypes.c_void_p(out.data_ptr()), h,
                                   ctypes.byref(flop))
        if st != 0:
            raise RuntimeError("umi_diag_fma_peak failed (%d)" % st)
    for _ in range(3):
        launch()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(launches):
        launch()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / launches
    tf = flop.value / (ms * 1e-3) / 1e12
    log("measured scalar FP32 FMA peak: %.1f TFLOP/s (%.3f ms per launch)" % (tf, ms))
    return tf


SERVE_POOL = 1000  # distinct curves drawn like the mixed workload, cycled by arrivals


def serve_sweep(rates, seconds, budget_gb, log, check_oracle=True, oracle_every=50,
                copy_threads=4, scheduler="native"):
    """Open-loop serving: Poisson arrivals (rate curves/s) of curves drawn like
    the mixed workload, device-memory budget `budget_gb`; latency from the
    scheduled arrival to the result in host memory.  `scheduler`: "native"
    (the library's serving loop) or "python" (the same loop in Python over the
    library's plan and copy calls)."""
    import synth
    from paper_2604_06602_amd.serve import (BYTES_PER_SAMPLE, GpuExecutor, NativeServer, Server,
                                            run_open_loop)
    log("drawing %d serving curves" % SERVE_POOL)
    pool = [synth.curve_for(4, i) for i in range(SERVE_POOL)]
    capacity = int(budget_gb * 1e9) // BYTES_PER_SAMPLE
    results = []
    if scheduler == "native":
        ex = None
        srv = NativeServer(capacity, max_curves=4096, max_W=721, copy_threads=copy_threads)
    else:
        ex = GpuExecutor(capacity, max_curves=4096, max_W=721, copy_threads=copy_threads)
        srv = Server(ex)
    for i in range(8):  # warm up: capture both graph slots, touch the pinned pool
        srv.submit(*pool[i]).result()
    for rate in rates:
        arrivals = synth.poisson_arrivals(rate, seconds, seed=int(rate))
        srv.reset_stats()
        keep = (lambda i: i % oracle_every == 0) if check_oracle else None
        summary, kept = run_open_loop(
            srv, pool, arrivals, keep,
            progress=lambda n, sec: log("rate %g/s: %d submitted after %.0f s" % (rate, n, sec)))
        entry = {"rate_curves_per_s": rate, "seconds": seconds, "requests": int(arrivals.size),
                 "budget_gb": budget_gb, "scheduler": scheduler, **summary}
        if check_oracle and kept:
            import oracle
            oracle.build(force=False)
            rng = np.random.default_rng(0)
            worst, compared, nan_mismatch = 0.0, 0, 0
            for i, (ci, res) in kept.items():
                f, t, W = pool[ci]
                idx = np.unique(rng.integers(0, f.size, 64))
                o_tr, _ = oracle.detrend_at(f, t, W, idx)
                ok = ~np.isnan(o_tr)
                g = res[idx]
                nan_mismatch += int(np.count_nonzero(np.isnan(g) != ~ok))
                if ok.any():
                    rel = np.abs(g[ok] - o_tr[ok]) / np.abs(o_tr[ok])
                    worst = max(worst, float(np.max(np.where(np.isnan(rel), np.inf, rel))))
                    compared += int(ok.sum())
            entry["oracle_checked_requests"] = len(kept)
            entry["oracle_compared_samples"] = compared
            entry["nan_pattern_mismatches"] = nan_mismatch
            entry["max_rel_err_vs_fp64_oracle"] = worst
        log("rate %g/s: p50 %.2f ms, p99 %.2f ms, %.0f curves/s, %d steps"
            % (rate, entry["p50_ms"] or -1, entry["p99_ms"] or -1, entry["curves_per_s"] or -1,
               entry["steps"]))
        results.append(entry)
    srv.close()
    del ex, srv
    return {"metric": "serving latency (open-loop Poisson arrivals, mixed curves)",
            "unit": "ms", "rates": results}


def batch_prefix(batch, n):
    import synth
    return synth.lightcurves.pack([batch.curve(i) for i in range(n)])


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", type=int, choices=[0, 1, 2, 3], default=1,
                    help="0: one 20k-sample TESS curve, W=361 (per-call latency); "
                         "1: 1000x18k TESS batch, W=361 (headline); 2: 2000 Kepler-like curves "
                         "of 40k-70k, W=25; 3: 10,000 mixed curves of 1k-120k, W in "
                         "{25,121,361,721}, 5%% NaN gaps")
    ap.add_argument("--mode", choices=["persistent", "per-curve"], default="persistent")
    ap.add_argument("--no-compare-per-curve", action="store_true",
                    help="skip timing one launch per curve on the same batch (the comparison "
                         "runs by default on workloads 1-3)")
    ap.add_argument("--tuning", default="auto",
                    help="'auto' (the committed tuning table for this GPU, if any), 'none' "
                         "(built-in defaults) or a table file")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--serve", action="store_true",
                    help="serving sweep instead: open-loop Poisson arrivals of mixed curves "
                         "at each --rates value (curves/s) for --serve-seconds each")
    ap.add_argument("--rates", default="100,300,1000,3000,10000,20000")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--copy-threads", type=int, default=4,
                    help="host threads for pinned staging and result copies in serving")
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-scheduler", choices=["native", "python"], default="native",
                    help="serving loop: the library's native scheduler, or the Python one")
    ap.add_argument("--quantize", type=float, default=0.0, metavar="STEP",
                    help="round the workload's flux to multiples of STEP (ties in every window; "
                         "for timing the tie handling)")
    ap.add_argument("--no-serve-leg", action="store_true",
                    help="skip the short serving measurement of the default run")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (to scale "
                         "HBM byte counters) and exit")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU: the estimate would shard over curves with no "
              "exchange step, but only single-GPU runs are implemented; --gpus %d is not "
              "supported" % args.gpus, file=sys.stderr)
        return 2

    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "launches": 5}))
        return 0

    import paper_2604_06602_amd as umi
    import synth

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    if args.serve:
        rates = [float(r) for r in args.rates.split(",")]
        out = serve_sweep(rates, args.serve_seconds, args.budget_gb, log,
                          check_oracle=not args.no_cpu_baseline, copy_threads=args.copy_threads,
                          scheduler=args.serve_scheduler)
        print(json.dumps(out), flush=True)
        return 0

    log("generating workload %d" % args.workload)
    batch = synth.config_batch(args.workload)
    if args.quantize > 0:
        # heavy ties: every flux a multiple of the step (NaN stays NaN)
        batch.flux[:] = (np.round(batch.flux.astype(np.float64) / args.quantize)
                         * args.quantize).astype(np.float32)
        log("flux quantised to multiples of %g" % args.quantize)
    alpha, c, iters = 2.0, 5.0, 5
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    flux = torch.from_numpy(batch.flux).to(dev)
    tim = torch.from_numpy(batch.time).to(dev)
    trend = torch.empty_like(flux)
    lengths = batch.lengths
    Ws = batch.W
    mode = umi.MODE_PERSISTENT if args.mode == "persistent" else umi.MODE_PER_CURVE
    stream = torch.cuda.current_stream()
    tuning = "built-in defaults"
    if args.tuning == "auto":
        from paper_2604_06602_amd import autotune
        if autotune.apply():
            tuning = "tuning table " + autotune.cache_key()
    elif args.tuning.endswith(".json"):
        from paper_2604_06602_amd import autotune
        if not autotune.apply(args.tuning):
            raise SystemExit("no tuning entry for %s in %s" % (autotune.cache_key(), args.tuning))
        tuning = "tuning table %s from %s" % (autotune.cache_key(), args.tuning)
    elif args.tuning != "none":
        umi.set_tuning(open(args.tuning).read())
        tuning = "tuning table " + args.tuning

    def step(ev0=None, ev1=None, m=None):
        umi.detrend_batch_into(flux, tim, lengths, Ws, trend, None, alpha, c, iters,
                               umi.LaunchOptions(mode=mode if m is None else m,
                                                 main_start=ev0, main_stop=ev1),
                               stream)

    # host-side preparation first, so the GPU does not idle between the
    # warm-up and the timed steps (its clock drops when idle)
    nwin = window_sizes(batch)
    window_samples = int(nwin.sum())
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:  # create the HIP events before handing them to the library
        a.record(stream)
        b.record(stream)
    t_start = torch.cuda.Event(enable_timing=True)
    t_stop = torch.cuda.Event(enable_timing=True)
    step()
    torch.cuda.synchronize()
    windows = int(torch.isfinite(trend).sum().item())
    if int((nwin > 0).sum()) != windows:
        raise RuntimeError("host window count %d != finite outputs %d" % ((nwin > 0).sum(), windows))

    log("warmup %d, then timing %d steps" % (args.warmup, args.steps))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for a, b in evs:
        step(a, b)
    t_stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_stop)
    ms_step = total_ms / args.steps
    main_each = [a.elapsed_time(b) for a, b in evs]
    main_ms = float(np.mean(main_each))
    value = windows / (ms_step * 1e-3)
    # algorithmic work: Phase 2 at 3 and each Phase 3 iteration at 8 FLOP per window sample
    flop_launch = window_samples * (3 + 8 * iters)
    achieved = flop_launch / (main_ms * 1e-3) / 1e12
    log("step %.3f ms (main %.3f ms), wall %.3f s" % (ms_step, main_ms, wall))
    log("main kernel per step (ms): " + " ".join("%.3f" % v for v in main_each))
    fma_peak = measured_fma_peak(torch, stream, log)

    per_curve = None
    if not args.no_compare_per_curve and args.workload != 0:
        other = umi.MODE_PER_CURVE if mode == umi.MODE_PERSISTENT else umi.MODE_PERSISTENT
        k = max(3, args.steps // 4)
        for _ in range(2):
            step(m=other)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(k):
            step(m=other)
        b.record(stream)
        torch.cuda.synchronize()
        oms = a.elapsed_time(b) / k
        name = "per-curve" if other == umi.MODE_PER_CURVE else "persistent"
        per_curve = {"mode": name, "ms_per_step": oms, "value": windows / (oms * 1e-3),
                     "steps": k, "speedup_of_%s" % args.mode: oms / ms_step}
        log("%s: %.3f ms per step" % (name, oms))

    latency = None
    if args.workload == 0:
        # one curve is launch-bound. The timed steps above carry a pair of
        # timing events around each estimate kernel, which on this scale cost
        # several microseconds per call; device time per call is also timed
        # over back-to-back calls without them. Then whole calls, launch to
        # result on the device (host clock around the call and a stream
        # synchronise).
        k = max(100, args.steps)
        for _ in range(10):
            step()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(k):
            step()
        b.record(stream)
        torch.cuda.synchronize()
        dev_us = a.elapsed_time(b) / k * 1e3
        walls = []
        for _ in range(max(50, args.steps)):
            w0 = time.perf_counter()
            step()
            stream.synchronize()
            walls.append(time.perf_counter() - w0)
        walls = np.array(walls) * 1e6
        latency = {"call_to_done_us_p50": float(np.percentile(walls, 50)),
                   "call_to_done_us_p99": float(np.percentile(walls, 99)),
                   "device_us_per_call": dev_us, "device_calls": k,
                   "device_us_per_call_with_kernel_events": ms_step * 1e3,
                   "calls": int(walls.size)}
        log("one curve: %.1f us device per call (%.1f with kernel timing events), "
            "%.1f us call to done (p50)"
            % (dev_us, ms_step * 1e3, latency["call_to_done_us_p50"]))

    wl = WORKLOADS[args.workload]
    out = {
        "metric": METRIC if args.workload == 1 else "window-estimates/s (%s)" % wl,
        "value": value,
        "unit": "window-estimates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl + ("_quantized_%g" % args.quantize if args.quantize > 0 else ""),
                   "curves": int(batch.n_curves),
                   "samples": int(batch.n_samples),
                   "W": sorted(set(int(w) for w in batch.W)), "alpha": alpha, "c": c,
                   "iters": iters, "windows": windows, "mode": args.mode, "tuning": tuning,
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "kernel": "umi_main_kernel",
                     "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": counted_traffic(args.workload) if args.quantize == 0 else None,
                     "target_frac": TARGET_FRAC,
                     "target_met": achieved / PEAK_FP32_TFLOPS >= TARGET_FRAC,
                     "traffic_unit": "bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-calibrated)",
                     "avg_launch_ms": main_ms, "flop_per_launch": flop_launch,
                     "window_samples_per_launch": window_samples,
                     "flop_per_window_sample": 3 + 8 * iters,
                     "measured_fma_peak": fma_peak,
                     "frac_of_measured_fma_peak": achieved / fma_peak},
    }
    if per_curve is not None:
        out["comparison"] = per_curve
    if latency is not None:
        out["latency"] = latency
    if not args.no_serve_leg:
        log("serving leg: 2000 curves/s for 3 s")
        del flux, tim, trend
        torch.cuda.empty_cache()
        # every 50th request is checked against the FP64 oracle after the run
        out["serve"] = serve_sweep([2000.0], 3.0, args.budget_gb, log, check_oracle=True,
                                   scheduler=args.serve_scheduler)["rates"][0]
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        if args.workload in (2, 3):
            # the first 100 curves, extrapolated to the whole workload
            out["cpu_baseline"] = cpu_baseline(batch, first_curves=100, total_windows=windows)
        else:
            out["cpu_baseline"] = cpu_baseline(batch, args.cpu_budget, total_windows=windows)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
