"""Throughput of the likelihood + gradient evaluation on one MI355X.

Workload: the N = 1000 balanced network (800 E / 200 I, fixed in-degree 100,
J_E = +0.2, J_I = -1.0, base rates U[5, 10] Hz, tau = 10 ms) recorded for
3600 s on a 1 ms grid (B = 3.6e6 bins), synthetic, seed 0.

A step is one evaluation of L and its full gradient (dL/dJ, dL/dmu) at the
current parameters: kernel U (V = J x, W = exp V, row sums), kernel G (W x^T
split over time), the FP64 reductions and the assembly.  The trace x depends
on the spikes and tau only; in BF16 it is resident by default (built once per
tau, "trace": "resident"), otherwise ("--trace recompute", and in FP32/FP64)
both contractions rebuild its tiles from the spike masks inside the step.
The per-recording and per-tau set-up (spike ingest, carries, spike term,
resident trace) runs once before the timed region and is reported as
setup_ms; after the timed evaluations the ascent reconstructs the network
from J = 0: BF16 to its stopping test, then BF16 with a two-term J (the
default --polish) to the FP64 oracle's optimum (reconstruct_s, with the
misclassification rate of the fitted weights against the generating ones;
reconstruct_bf16_only_s is the first part alone).
value = B * N^2 / (seconds per step), in bins*N^2/s.

Other workloads (--workload): batch64 (64 recordings evaluated together),
events (the same recording in continuous time), reconstruct (BF16 ascent and
its continuation to the FP64 oracle's optimum, timed and classified).

Prints one JSON line.  N > 1 GPUs is not supported (one-GPU build).
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

PEAK = {"fp8": 5.0e15, "bf16": 2.5e15, "fp32": 157.3e12, "fp64": 78.6e12}  # dense MFMA, flop/s
HBM_PEAK = 8.0e12


def gemm_source_hash() -> str:
    """Hash of the sources of the resident-trace kernels U and G (the kernels
    the committed counter summary covers)."""
    h = hashlib.sha1()
    for f in ("gemm_res.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_1502_04993_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def traffic_from_profile(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a copy of known size), if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_kernels_U_G_balanced_n1000_bf16.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != gemm_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def time_steps(ctx, steps: int, warmup: int):
    """Seconds per evaluation of L and the full gradient; the gradient stays in
    device memory (where the ascent consumes it), L comes back to the host."""
    import torch
    import paper_1502_04993_amd as G
    gJ = torch.empty((ctx.N, ctx.N), dtype=torch.float64, device="cuda")
    gmu = torch.empty(ctx.N, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        G.glmr_eval(ctx.handle, None, gJ, gmu)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ll, _ = G.glmr_eval(ctx.handle, None, gJ, gmu)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, {"ll": ll}


def kernel_times(ctx, reps: int = 2):
    ctx.prof_reset()
    ctx.prof(True)
    import torch
    import paper_1502_04993_amd as G
    gJ = torch.empty((ctx.N, ctx.N), dtype=torch.float64, device="cuda")
    gmu = torch.empty(ctx.N, dtype=torch.float64, device="cuda")
    for _ in range(reps):
        G.glmr_eval(ctx.handle, None, gJ, gmu)
    out = ctx.prof_get()
    ctx.prof(False)
    return {k: (ms / reps, n // reps) for k, (ms, n) in out.items()}


def golden_row_errors(ctx, rec, prec):
    """Errors of the context's evaluation on the sampled rows that the FP64
    oracle evaluated over the whole recording (tests/golden/config2_grid_rows.json,
    written by a script that calls only the oracle): the stored rounded weight
    rows are set (the others keep the simulated values; L is separable over
    rows), one evaluation, and the relative errors of L_i (largest over the
    rows) and of the gradient rows (dL/dmu_i, dL/dJ_i.) as a 2-norm and
    element-wise (largest error over the largest entry)."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "config2_grid_rows.json")
    if rec.n_bins != 3_600_000 or not os.path.exists(path):
        return None
    gold = json.load(open(path))
    rows = gold["rows"]
    pt = gold["points"]["fp8" if prec == "fp8" else "bf16"]
    J = rec.J.copy()
    J[rows] = np.array([[float(v) for v in r] for r in pt["J_rows"]])
    ctx.set_params(J, rec.mu)
    r = ctx.eval(grad=True)
    ll = np.array([float(v) for v in pt["ll_rows"]])
    g = np.concatenate([r["gmu"][rows], r["gJ"][rows].ravel()])
    gr = np.concatenate([np.array([float(v) for v in pt["gmu"]]),
                         np.array([[float(v) for v in row] for row in pt["gJ"]]).ravel()])
    return {"rows": rows, "ll_row_rel_err": float(np.max(np.abs(r["ll_rows"][rows] - ll) / np.abs(ll))),
            "grad_rel_err": float(np.linalg.norm(g - gr) / np.linalg.norm(gr)),
            "grad_max_err": float(np.max(np.abs(g - gr)) / np.max(np.abs(gr)))}


def cpu_baseline(rec, sample_bins: int):
    """The FP64 oracle on a bounded sample of the same workload (the first
    `sample_bins` bins), scaled to bins*N^2/s."""
    import numpy as np
    from oracle import glm_oracle as O
    n_threads = os.cpu_count() or 1
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        n_threads = max(i.get("num_threads", 1) for i in info if i.get("user_api") == "blas")
    except Exception:
        pass
    N = rec.n_neurons
    t0 = time.perf_counter()
    O.loglik(rec.bins, rec.neurons, N, rec.n_bins, rec.dt, rec.tau, rec.J, rec.mu,
             bin_range=(0, sample_bins))
    dt = time.perf_counter() - t0
    return {"value": sample_bins * N * N / dt, "unit": "bins*N^2/s", "cores": int(n_threads),
            "kind": "oracle",
            "sample": f"FP64 L + gradient over bins [0, {sample_bins}) of the same recording "
                      f"(N = {N}); {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp8", "fp32", "fp64"])
    ap.add_argument("--bins", type=int, default=3_600_000)
    ap.add_argument("--trace", default="auto", choices=["auto", "resident", "recompute"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shapes")
    ap.add_argument("--workload", default="balanced_n1000",
                    choices=["balanced_n1000", "batch64", "events", "reconstruct", "cv"],
                    help="batch64: 64 recordings of uneven N and T (balanced and synfire), "
                         "evaluated together (grouped launches); events: the balanced N = 1000 "
                         "recording in continuous time (event grid, Ei integrals); reconstruct: "
                         "time to reconstruct the N = 1000 network (BF16 fit from zero, FP32 polish) "
                         "and the misclassification rate against the generated weights; cv: a "
                         "cross-validation scan over tau on the N = 500, 600 s recording")
    ap.add_argument("--fit-max-iter", type=int, default=400, help="reconstruct: BF16 ascent cap")
    ap.add_argument("--polish-iter", type=int, default=0,
                    help="cap of the continuation of the BF16 ascent (reconstruct and the default run); "
                         "0: 400 for bf16j2, 60 for fp32")
    ap.add_argument("--polish", default="bf16j2", choices=["bf16j2", "fp32", "none"],
                    help="precision that continues the BF16 ascent to the oracle's optimum: bf16j2 (BF16 "
                         "with J as two BF16 terms, the trace kept) or fp32")
    ap.add_argument("--cpu-sample-events", type=int, default=12000,
                    help="events: network events of the oracle's bounded sample")
    ap.add_argument("--n-rec", type=int, default=64, help="batch64: number of recordings")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--delays", default="",
                    help="d,d_self: transmission delays in bins (Eq. (15)) on the default workload")
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8 comparison line")
    ap.add_argument("--cpu-sample-bins", type=int, default=1_572_864)
    ap.add_argument("--fit-iters", type=int, default=400,
                    help="cap of the ascent from J = 0 timed after the evaluations (0: skip); "
                         "the fitted weights are classified against the generating ones")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run a device-to-device copy of this many MiB (a known-size "
                         "kernel for calibrating HBM byte counters)")
    args = ap.parse_args()
    if args.polish_iter <= 0:
        args.polish_iter = 60 if args.polish == "fp32" else 400
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "see DESIGN.md for how the evaluation would shard", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_1502_04993_amd as G

    torch.cuda.init()
    if args.workload == "batch64":
        bench_batch(args, G, torch)
        return
    if args.workload == "events":
        bench_events(args, G, torch)
        return
    if args.workload == "reconstruct":
        bench_reconstruct(args, G, torch)
        return
    if args.workload == "cv":
        bench_cv(args, G, torch)
        return
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    rec = synth.cached("config2", seed=0, B=args.bins)
    N, B = rec.n_neurons, rec.n_bins
    units = float(B) * N * N

    delays = tuple(int(v) for v in args.delays.split(",")) if args.delays else (0, 0)

    def run(prec):
        ctx = G.Context(N, B, rec.dt, precision=prec, trace=args.trace if prec == "bf16" else "auto")
        t0 = time.perf_counter()
        if delays != (0, 0):
            ctx.set_delays(*delays)
        ctx.set_spikes(rec.bins, rec.neurons)
        ctx.set_kernel(rec.tau)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        ctx.set_params(rec.J, rec.mu)
        tiles = ctx.autotune() if prec in ("bf16", "fp8") and not args.no_tune else (-1, -1)
        sec, r = time_steps(ctx, args.steps, args.warmup)
        kt = kernel_times(ctx)
        err = golden_row_errors(ctx, rec, prec) if delays == (0, 0) else None
        ctx.set_params(rec.J, rec.mu)
        return ctx, setup, sec, r, kt, tiles, err

    def dominant(kt, prec):
        """Dominant contraction of a step and its roofline against the mode's MFMA peak."""
        dom = max(("kernel_U", "kernel_G"), key=lambda k: kt.get(k, (0, 0))[0])
        ms_total, launches = kt[dom]
        per_launch_s = ms_total / 1e3 / launches
        achieved = 2.0 * N * N * B / launches / per_launch_s  # 2 flops per bin*N^2 per contraction
        return dom, launches, per_launch_s, achieved, PEAK[prec]

    ctx, setup, sec, r, kt, tiles, err = run(args.precision)
    q = ctx.query()
    dom, launches, per_launch_s, achieved, peak = dominant(kt, args.precision)
    traffic = traffic_from_profile(dom) if args.precision == "bf16" and q["trace_resident"] else None
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                "kernel": dom, "launch_ms": per_launch_s * 1e3, "launches_per_step": launches,
                "issued_frac": achieved * (q["n_pad"] / N) ** 2 / peak,
                "per_kernel_ms": {k: v[0] for k, v in kt.items()}}

    # the reconstruction: per-row L-BFGS ascent from J = 0 to its stopping test,
    # then the continuation that brings the fit to the FP64 oracle's optimum
    # (the fit the classification test compares with the oracle's rows), then
    # the E/I/none classification of the fitted weights (Sec. 3.3)
    fit_info = None
    if args.fit_iters > 0:
        from paper_1502_04993_amd.classify import classify, misclassification
        t0 = time.perf_counter()
        fr = ctx.fit(max_iter=args.fit_iters, from_zero=True)
        t_fit = time.perf_counter() - t0
        Jf, _, _ = ctx.get_params()
        m0 = misclassification(classify(Jf), rec.J)
        fit_info = {"iters": fr["iters"], "evals": fr["evals"], "converged": fr["converged"],
                    "rows_converged": fr["rows_converged"], "seconds": t_fit,
                    "iters_per_s": fr["iters"] / t_fit, "mer": m0["mer"], "mer_n2": m0["mer_n2"]}
        if args.polish_iter > 0 and args.precision == "bf16" and args.polish != "none":
            t1 = time.perf_counter()
            ctx.set_precision(args.polish)
            pr = ctx.fit(max_iter=args.polish_iter, keep_history=True)
            ctx.set_precision(args.precision)
            t_pol = time.perf_counter() - t1
            Jp, _, _ = ctx.get_params()
            m = misclassification(classify(Jp), rec.J)
            fit_info.update({"polish": args.polish, "polish_iters": pr["iters"],
                             "polish_rows_converged": pr["rows_converged"], "polish_seconds": t_pol,
                             "seconds_bf16_only": t_fit, "mer_bf16_only": m0["mer"],
                             "seconds": t_fit + t_pol, "mer": m["mer"], "mer_n2": m["mer_n2"]})
    ctx.close()

    extra = {}
    if not args.no_fp8 and args.precision == "bf16" and delays[0] == delays[1]:  # FP8 needs d_self = d
        c8, setup8, sec8, r8, kt8, tiles8, err8 = run("fp8")
        c8.close()
        dom8, _, pl8, ach8, peak8 = dominant(kt8, "fp8")
        extra.update({"fp8_value": units / sec8, "fp8_ms_per_step": sec8 * 1e3,
                      "fp8_tile_shapes": list(tiles8), "fp8_errors": err8,
                      "fp8_roofline": {"bound": "mfma", "achieved": ach8 / 1e12, "peak": peak8 / 1e12,
                                       "unit": "TFLOP/s", "frac": ach8 / peak8, "kernel": dom8,
                                       "launch_ms": pl8 * 1e3}})
    if not args.no_fp32 and args.precision != "fp32":
        c32, setup32, sec32, r32, kt32, _, err32 = run("fp32")
        c32.close()
        extra.update({"fp32_value": units / sec32, "fp32_ms_per_step": sec32 * 1e3,
                      "bf16_over_fp32": sec32 / sec, "fp32_errors": err32})

    out = {
        "metric": "LL+grad throughput (bins*N^2/s) at N=1000; BF16 vs FP32 at stated grad error",
        "value": units / sec,
        "unit": "bins*N^2/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "balanced_n1000_indeg100_t3600s_dt1ms", "n_neurons": N,
                   "n_bins": B, "n_spikes": rec.n_spikes, "precision": args.precision,
                   "chunk_bins": q["chunk_bins"], "n_pad": q["n_pad"],
                   "trace": "resident" if q["trace_resident"] else "recompute",
                   "tile_shapes": list(tiles), "delays_bins": list(delays)},
        "roofline": roofline,
        "errors": err,
        "grad_rel_err": err["grad_rel_err"] if err else None,
        "setup_ms": setup * 1e3,
        "ll": r["ll"],
        "fit": fit_info,
        "reconstruct_s": fit_info["seconds"] if fit_info else None,
        "reconstruct_bf16_only_s": fit_info.get("seconds_bf16_only", fit_info["seconds"]) if fit_info else None,
    }
    out.update(extra)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(rec, min(args.cpu_sample_bins, B))
    print(json.dumps(out))


def cpu_baseline_events(times, neurons, N, tau, J, mu, n_events):
    """The FP64 oracle's continuous-time L + gradient over the first n_events
    network events (the window [0, t of event n_events)), scaled to slots*N^2/s."""
    from oracle import glm_oracle as O
    n_threads = os.cpu_count() or 1
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        n_threads = max(i.get("num_threads", 1) for i in info if i.get("user_api") == "blas")
    except Exception:
        pass
    T1 = float(times[n_events])
    t, n = times[:n_events], neurons[:n_events]
    lists = [t[n == j] for j in range(N)]
    t0 = time.perf_counter()
    O.continuous_eval(lists, 0.0, T1, tau, J, mu)
    dt = time.perf_counter() - t0
    return {"value": (n_events + 1) * N * N / dt, "unit": "slots*N^2/s", "cores": int(n_threads),
            "kind": "oracle",
            "sample": f"FP64 continuous-time L + gradient over the first {n_events} events of the same "
                      f"recording (window [0, {T1:.3f}) s, N = {N}); {dt:.1f} s"}


def bench_events(args, G, torch):
    """Continuous-time L + gradient on the event grid: the balanced N = 1000
    recording with every spike placed uniformly inside its 1 ms bin, so the
    slots are the intervals between ~2.7e7 network events.  A step is one
    evaluation; value = slots * N^2 / (seconds per step)."""
    import synth
    prec = args.precision if args.precision in ("fp64", "fp32", "bf16") else "fp64"
    rec = synth.cached("config2", seed=0, B=args.bins)
    N = rec.n_neurons
    times, neu = synth.event_times(rec, seed=0)
    T0, T1 = 0.0, rec.T
    print(f"[events] {times.shape[0]} events ready", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ctx = G.Context.from_events(N, times, neu, T0, T1, precision=prec,
                                trace=args.trace if prec == "bf16" else "auto")
    ctx.set_kernel(rec.tau)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    slots = ctx.B
    ctx.set_params(rec.J, rec.mu)
    tiles = ctx.autotune() if prec == "bf16" and not args.no_tune else (-1, -1)
    print(f"[events] context ready: {slots} slots, setup {setup:.2f} s, tile shapes {tiles}",
          file=sys.stderr, flush=True)
    sec, r = time_steps(ctx, args.steps, args.warmup)
    kt = kernel_times(ctx, reps=1)
    q = ctx.query()
    ctx.close()
    dom = max(("kernel_U", "kernel_G"), key=lambda k: kt.get(k, (0, 0))[0])
    ms_total, launches = kt[dom]
    per_launch_s = ms_total / 1e3 / launches
    achieved = 2.0 * N * N * slots / launches / per_launch_s
    # FP64 and FP32 modes run both contractions on the FP64 MFMA; BF16 on the BF16 one
    peak = PEAK["bf16"] if prec == "bf16" else PEAK["fp64"]
    units = float(slots) * N * N
    out = {
        "metric": "continuous-time LL+grad throughput (slots*N^2/s) at N=1000",
        "value": units / sec, "unit": "slots*N^2/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[prec],
        "data": "synthetic",
        "config": {"workload": "balanced_n1000_indeg100_t3600s_event_grid", "n_neurons": N,
                   "n_events": int(times.shape[0]), "n_slots": slots, "precision": prec,
                   "chunk_slots": q["chunk_bins"], "n_pad": q["n_pad"], "trace_resident": q["trace_resident"],
                   "tile_shapes": list(tiles)},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None, "kernel": dom,
                     "launch_ms": per_launch_s * 1e3, "launches_per_step": launches,
                     "per_kernel_ms": {k: v[0] for k, v in kt.items()}},
        "setup_ms": setup * 1e3, "ll": r["ll"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_events(times, neu, N, rec.tau, rec.J, rec.mu,
                                                  min(args.cpu_sample_events, times.shape[0] - 1))
    print(json.dumps(out))


def bench_cv(args, G, torch):
    """Cross-validation scan over the kernel time constant (Sec. 3.2, Fig. 4)
    and the penalty strength (Sec. 2.5): the N = 500 balanced recording of
    600 s (true tau = 8 ms) split in halves, one batched fit from J = 0 per
    penalty level over the tau grid, each fit scored on the held-out half.
    Value: the wall time of the whole scan, context set-up included (the
    spikes start on the host)."""
    from paper_1502_04993_amd.cv import cv_scan
    import synth
    rec = synth.cached("config4", seed=0)
    taus = [0.004, 0.006, 0.008, 0.012, 0.016]
    prec = args.precision if args.precision in ("fp32", "bf16", "fp64") else "bf16"
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alphas = (0.0, 2.0)  # unpenalised, and the smooth epsilon-l1 penalty of Eq. (16)-(17)
    res = cv_scan(rec.bins, rec.neurons, rec.n_neurons, rec.n_bins, rec.dt, taus, alphas=alphas, precision=prec)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    best = res.best()
    iters = [[res.reports[(a, k)]["iters"] for k in range(len(taus))] for a in range(len(alphas))]
    out = {
        "metric": "cross-validation scan over tau (5 points) and alpha (2), N=500, 600 s",
        "value": sec, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": sec * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[prec], "data": "synthetic",
        "config": {"workload": "balanced_n500_indeg50_t600s_tau8ms_cv", "n_neurons": rec.n_neurons,
                   "n_bins": rec.n_bins, "taus_s": taus, "alphas": list(alphas), "train_frac": 0.5, "precision": prec},
        "roofline": None,
        "best_alpha": best[0], "best_tau_s": best[1], "true_tau_s": rec.tau,
        "mean_row_peak_tau_s": res.mean_row_peak_tau(0),
        "validation_ll": [[float(v) for v in row] for row in res.val], "fit_iters": iters,
    }
    print(json.dumps(out))


def bench_reconstruct(args, G, torch):
    """Time to reconstruct the N = 1000 network: BF16 ascent from J = 0, mu = 0
    to its stopping test, then FP32 evaluations from the BF16 optimum, then
    the E/I/none classification of the fitted weights (Sec. 3.3) and its
    error rate against the generating ones (Eq. (20)).  The timed region
    starts with the spikes resident (ingest and the per-tau set-up are
    reported apart)."""
    import numpy as np
    from paper_1502_04993_amd.classify import classify, misclassification
    import synth
    rec = synth.cached("config2", seed=0, B=args.bins)
    N, B = rec.n_neurons, rec.n_bins
    t0 = time.perf_counter()
    ctx = G.Context(N, B, rec.dt, precision="bf16")
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    print(f"[reconstruct] set-up {setup:.2f} s", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    rep = ctx.fit(max_iter=args.fit_max_iter, from_zero=True)
    J16, _, _ = ctx.get_params()
    t_bf16 = time.perf_counter() - t1
    lab16 = classify(J16)
    m16 = misclassification(lab16, rec.J)
    print(f"[reconstruct] BF16 ascent {t_bf16:.2f} s, {rep['iters']} steps, MER {m16['mer']:.4%}",
          file=sys.stderr, flush=True)
    t2 = time.perf_counter()
    pol = None
    if args.polish_iter > 0 and args.polish != "none":
        ctx.set_precision(args.polish)
        pol = ctx.fit(max_iter=args.polish_iter, from_zero=False, keep_history=True)
        ctx.set_precision("bf16")
    J, mu, _ = ctx.get_params()
    t_pol = time.perf_counter() - t2
    ctx.close()
    t3 = time.perf_counter()
    lab = classify(J)
    m = misclassification(lab, rec.J)
    t_cls = time.perf_counter() - t3
    off = ~np.eye(N, dtype=bool)
    out = {
        "metric": f"time to reconstruct N=1000 (BF16 ascent + {args.polish} continuation)",
        "value": t_bf16 + t_pol, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": (t_bf16 + t_pol) * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "balanced_n1000_indeg100_t3600s_dt1ms", "n_neurons": N, "n_bins": B,
                   "n_spikes": rec.n_spikes, "fit_max_iter": args.fit_max_iter, "polish": args.polish,
                   "polish_iter": args.polish_iter},
        "bf16": {"seconds": t_bf16, "fit": rep, "mer": m16["mer"], "mer_n2": m16["mer_n2"],
                 "errors": m16["errors"]},
        "polish": {"seconds": t_pol, "fit": pol},
        "setup_s": setup, "classify_s": t_cls,
        "mer": m["mer"], "mer_n2": m["mer_n2"], "errors": m["errors"],
        "labels_changed_by_polish": int((lab[off] != lab16[off]).sum()),
        "max_abs_J_change_by_polish": float(np.abs(J - J16).max()),
        "max_abs_J_error": float(np.abs(J - rec.J).max()),
    }
    print(json.dumps(out))


def bench_batch(args, G, torch):
    """64 recordings (N ~ U{100..2000}, synfire half U{625..2000}; T ~ U[60, 600] s;
    even balanced, odd synfire), all evaluated by one batched call: the value is
    sum_r B_r N_r^2 over the seconds of one batched evaluation."""
    import synth
    sizes = synth.config5_sizes()[: args.n_rec]
    ctxs, units, nbins = [], 0.0, 0
    t_setup = time.perf_counter()
    for r, (kind, N, B, seed) in enumerate(sizes):
        rec = synth.config5_recording(kind, N, B, seed)
        c = G.Context(N, B, rec.dt, precision=args.precision)
        c.set_spikes_allow_silent(rec.bins, rec.neurons)
        c.set_kernel(rec.tau)
        c.set_params(rec.J, rec.mu)
        ctxs.append(c)
        units += float(B) * N * N
        nbins += B
        print(f"[batch64] recording {r} {kind} N={N} B={B} ready", file=sys.stderr, flush=True)
        del rec
    b = G.Batch(ctxs)
    tiles = b.autotune() if not args.no_tune else (-1, -1)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t_setup
    for _ in range(args.warmup):
        b.eval()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lls = b.eval()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    peak = PEAK[args.precision]
    achieved = 4.0 * units / sec
    out = {
        "metric": "LL+grad throughput (bins*N^2/s), recordings batched",
        "value": units / sec, "unit": "bins*N^2/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"batch{len(sizes)}_balanced_synfire_uneven_n_t", "n_recordings": len(sizes),
                   "sum_bins": nbins, "sum_bins_N2": units, "tile_shapes": list(tiles)},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "whole batched evaluation (4 sum B N^2 flop per evaluation)"},
        "setup_ms": setup * 1e3, "ll_sum": float(sum(lls)),
    }
    for c in ctxs:
        c.close()
    b.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
