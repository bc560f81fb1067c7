#!/usr/bin/env python3
"""Throughput of the MPI model operator pair A + A^T on one MI355X.

Workload (the headline shape): 256 x 256 grid, 53,856 Lissajous samples
(33 periods of 1632, 17:16 cycles), full-size Langevin kernel (R = 255, FFT
path with M = 512), float32, the ellipse-and-line phantom.  One pair is
s = A c followed by c' = A^T s, with every input resident in device memory.

`value` is the whole-job pair rate when `--batch` independent problems of that
shape are processed per call: a step is one call of the library's pair entry
(s = A c, then A^T s, for every problem of the batch).  After `--warmup`
untimed steps, `--runs` runs (default 5) of exactly `--steps` steps each are
timed and the median run gives the value; without `--steps` the step count
is chosen so that one run lasts at least `--run-seconds` (default 1 s).  The library splits such a
batch into problem ranges on side streams (two at 64 problems, four below 48),
and each range's transpose
follows its own forward with no join in between, as inside the library's
iteration.  The same pairs as a forward call then a transpose call are
reported under "separate_calls", the single-problem rate under
"single_problem".  Timed
steps are replayed from captured HIP graphs; HIP events on the launch stream
give the times.

Also reported: per-kernel durations (each stage launched alone through the
library's diagnostic entry point), the roofline of the dominant kernel, the
fraction of HBM peak for the algorithmic bytes of a pair (56 N^2 + 48 T), the
uneven 64-problem batch iteration against 64 sequential solves, the same
workload with the cosine interpolator, and the float64 CPU oracle timed on a
bounded sample of pairs on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0


def src_digest() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "paper_2505_22797_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


STAGE_NAMES = ("fwd_rows", "fwd_cols", "fwd_rows_gather", "adj_scatter_row", "adj_cols", "adj_rows")


def stage_bytes(name: str, n: int, m: int, t: int, elem: int = 4, spectra: float = 1.0) -> float:
    """Compulsory bytes of one launch of a stage for one problem: every input
    and output of the stage moved once (plan constants included).  spectra:
    copies of the kernel spectra per problem (1/B for a batch of B problems
    sharing one kernel, whose plan holds one copy)."""
    hh = m // 2 + 1
    cplx = 2 * elem
    samp = t * (4 * elem + 8)          # (fx, fy, vx, vy) and (base cell, time index)
    spec = spectra * elem * 3 * hh * hh
    return {
        "fwd_rows": elem * n * n + cplx * hh * n,
        "fwd_cols": cplx * hh * n + spec + 3 * cplx * n * hh,
        "fwd_rows_gather": 3 * cplx * n * hh + samp + 2 * elem * t,
        "adj_scatter_row": samp + 2 * elem * t + 3 * cplx * hh * n,
        "adj_cols": 3 * cplx * hh * n + spec + cplx * n * hh,
        "adj_rows": cplx * n * hh + elem * n * n,
    }[name]


def alg_stage_bytes(name: str, n: int, t: int, elem: int = 4) -> float:
    """The share of one stage in the algorithmic bytes of a pair (56 N^2 + 48 T
    in float32): c read 4N^2; the three-channel field G written and read,
    12N^2 each way; positions and velocities 16T and the signal 8T, once per
    direction; the transposed field G' written and read; c' written.  On the
    FFT path G and G' exist only as spectra, so the column stage that
    produces (consumes) a spectrum is credited with writing (reading) G (G')."""
    nn = elem * n * n
    samp = (4 * elem) * t + (2 * elem) * t      # r, v and s
    return {
        "fwd_rows": nn,
        "fwd_cols": 3 * nn,
        "fwd_rows_gather": 3 * nn + samp,
        "adj_scatter_row": samp + 3 * nn,
        "adj_cols": 3 * nn,
        "adj_rows": nn,
    }[name]


def counter_bytes(stage_names, batch: int):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by the copy
    calibration) of every stage with a counter record in profiles/ taken on
    the current kernel sources; None for a stage without one."""
    out = {}
    digest = src_digest()
    for name in stage_names:
        pmc = os.path.join(HERE, "profiles", f"k_{name}_headline_256_b{batch}_pmc.json")
        rec = json.load(open(pmc)) if os.path.exists(pmc) else {}
        out[name] = rec.get("hbm_bytes_per_launch") if rec.get("src_digest") == digest else None
    return out


def group_for(steps):
    """The largest graph size in (10, 8, 5, 4, 2, 1) that divides `steps`."""
    return next(g for g in (10, 8, 5, 4, 2, 1) if steps % g == 0)


def graph_time(fn, steps, group, warmup, runs=1):
    """Times `runs` runs of exactly `steps` calls of fn(), each replayed from a
    captured graph of `group` calls (group divides steps), after `warmup`
    untimed calls; HIP events on the launch stream bracket every run.
    Returns (median ms per call, steps per run, [ms per call of every run])."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(group):
            fn()
    g.replay()
    torch.cuda.synchronize()
    reps = max(1, (steps + group - 1) // group)
    per_run = []
    for _ in range(runs):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            g.replay()
        b.record()
        torch.cuda.synchronize()
        per_run.append(a.elapsed_time(b) / (reps * group))
    med = sorted(per_run)[len(per_run) // 2]
    return med, reps * group, per_run


def steps_for_seconds(fn, seconds, warmup):
    """Steps per run so that one run lasts at least `seconds` (a multiple of
    10, so that graphs of ten calls divide it), from a short timed probe.
    The probe's short graphs run a little slower per step than a long run,
    hence the 15 % margin."""
    ms, _, _ = graph_time(fn, 50, 10, warmup)
    return max(10, int(-(-1.15 * seconds * 1e3 / ms // 10)) * 10)


def stage_times(obj, c, s, reps):
    import torch
    out = {}
    for k, name in enumerate(obj.stages()):
        obj.launch_stage(k, 2, c, s)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        obj.launch_stage(k, reps, c, s)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        if ms > 0.002:      # stages of the path a plan does not use launch nothing
            out[name] = ms
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps per run (default: enough for runs of at least --run-seconds)")
    ap.add_argument("--runs", type=int, default=5, help="timed runs of the headline; the median is reported")
    ap.add_argument("--run-seconds", type=float, default=1.0)
    ap.add_argument("--aux-steps", type=int, default=100, help="timed steps of the secondary lines")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--graph-pairs", type=int, default=10)
    ap.add_argument("--ranges", type=int, default=-1,
                    help="problem ranges of the headline batch (-1: the build's count)")
    ap.add_argument("--stage-reps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-iter", action="store_true")
    ap.add_argument("--no-window", action="store_true")
    ap.add_argument("--no-cosine", action="store_true")
    ap.add_argument("--no-deconv", action="store_true")
    ap.add_argument("--no-two-stage", action="store_true")
    ap.add_argument("--no-kernel-per-problem", action="store_true",
                    help="skip the headline batch with a distinct kernel per problem")
    ap.add_argument("--two-stage-only", action="store_true",
                    help="only the two-stage reconstruction (for a kernel trace of its kernels)")
    ap.add_argument("--deconv-only", action="store_true",
                    help="only the deconvolution workload (for a kernel trace of its kernels)")
    ap.add_argument("--grad-only", action="store_true",
                    help="only the differentiation workload (for a kernel trace of its kernels)")
    ap.add_argument("--profile-batch", action="store_true",
                    help="only a few batched pairs plus a 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the operator runs on a single MI355X "
              "(sharding across GPUs is described in the design notes, not implemented)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    sys.path.insert(0, HERE)
    from paper_2505_22797_amd import mpik
    from paper_2505_22797_amd import synth as S

    P = S.headline()
    n, t = P.n, P.n_samples
    dev = torch.device("cuda:0")
    if args.grad_only:
        print(json.dumps({"differentiation": differentiation(S, dev)}))
        return 0
    if args.deconv_only:
        print(json.dumps({"deconvolution": deconvolution(mpik, S, dev, False)}))
        return 0
    if args.two_stage_only:
        print(json.dumps({"two_stage": two_stage(mpik, S, dev, False)}))
        return 0
    r = torch.tensor(S.to_f32(P.traj.r), dtype=torch.float32, device=dev)
    v = torch.tensor(S.to_f32(P.traj.v), dtype=torch.float32, device=dev)
    c1 = torch.tensor(P.c, dtype=torch.float32, device=dev)
    b_alg = 56 * n * n + 48 * t
    print(f"bench: headline 256^2 / {t} samples, batch {args.batch}", file=sys.stderr, flush=True)

    if args.profile_batch:
        return profile_batch(mpik, P, r, v, c1, max(1, args.batch), args.steps or 20)

    # ---- one problem per launch
    plan = mpik.Plan(n, P.h, P.radius, r, v)
    s1 = torch.empty((t, 2), dtype=torch.float32, device=dev)
    g1 = torch.empty((n, n), dtype=torch.float32, device=dev)

    def pair1():
        plan.forward(c1, s1)
        plan.adjoint(s1, g1)

    ms1, _, _ = graph_time(pair1, 10 * args.aux_steps, args.graph_pairs, args.warmup)
    st1 = stage_times(plan, g1, s1, args.stage_reps)
    print(f"bench: single problem {ms1 * 1e3:.1f} us/pair", file=sys.stderr, flush=True)

    # ---- B problems of the headline shape per launch
    B = max(1, args.batch)
    batch = mpik.Batch([(n, P.h, P.radius, r, v, "fft")] * B, tune=False)
    c_all = c1.reshape(-1).repeat(B).contiguous()
    s_all = torch.empty(batch.s_offsets[-1], dtype=torch.float32, device=dev)
    g_all = torch.empty(batch.c_offsets[-1], dtype=torch.float32, device=dev)
    ranges_default = batch.schedule()
    ranges = batch.schedule(args.ranges, c_all, s_all, g_all)

    def pairB():
        batch.pair(c_all, s_all, g_all)

    def pairB_separate():
        batch.forward(c_all, s_all)
        batch.adjoint(s_all, g_all)

    # the timed region: --runs runs of exactly --steps batch steps each, after
    # --warmup untimed ones; the median run gives the value
    steps = args.steps if args.steps else steps_for_seconds(pairB, args.run_seconds, args.warmup)
    msB, steps, runs = graph_time(pairB, steps, group_for(steps), args.warmup, runs=args.runs)
    msB_sep, _, runs_sep = graph_time(pairB_separate, steps, group_for(steps), args.warmup, runs=args.runs)
    stB = stage_times(batch, g_all, s_all, max(3, args.stage_reps // 4))
    pairs_per_s = B * 1e3 / msB
    # the same batch with a kernel of its own per problem (h differing in the
    # sixth digit), so that no two problems share kernel tables: B copies of
    # the spectra read per stage instead of one
    msB_d = None
    if not args.no_kernel_per_problem:
        batch_d = mpik.Batch([(n, P.h * (1.0 + 1e-6 * b), P.radius, r, v, "fft") for b in range(B)], tune=False)
        batch_d.schedule(ranges)
        msB_d, _, _ = graph_time(lambda: batch_d.pair(c_all, s_all, g_all), steps, group_for(steps), args.warmup)
        batch_d.close()
        del batch_d
        print(f"bench: batch {B}, a kernel per problem: {msB_d * 1e3:.1f} us/step, {B * 1e3 / msB_d:.0f} pairs/s",
              file=sys.stderr, flush=True)
    print(f"bench: batch {B} ({ranges} ranges): {msB * 1e3:.1f} us/step, {pairs_per_s:.0f} pairs/s", file=sys.stderr,
          flush=True)

    batch_fft = batch.info[0]["fft_size"]
    fft_stages = [k for k in stB if k in STAGE_NAMES]
    dom = max(fft_stages, key=stB.get)
    dom_alg = B * alg_stage_bytes(dom, n, t)
    achieved = dom_alg / (stB[dom] * 1e-3) / 1e9
    traffic = counter_bytes(fft_stages, B)
    known = [traffic[k] for k in fft_stages]
    counter_pair = sum(known) / B if all(x is not None for x in known) else None

    out = {
        "metric": "A+A^T applies/s at 256^2 grid, 53,856 samples (fraction of HBM peak)",
        "value": round(pairs_per_s, 1),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(msB, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "headline_256: N=256, T=53856 Lissajous 17:16, R=255 (FFT, M=512)",
                   "problems_per_step": B, "grid": n, "samples": t, "radius": plan.radius,
                   "fft_size": plan.fft_size, "conv_path": plan.conv_mode,
                   "problem_ranges": ranges, "ranges_by": "build" if args.ranges < 0 else "given",
                   "ranges_default": ranges_default},
        "timing": {"runs": len(runs), "steps_per_run": steps, "statistic": "median",
                   "ms_per_step_runs": [round(x, 5) for x in runs],
                   "spread": round((max(runs) - min(runs)) / msB, 4),
                   "run_seconds": round(msB * steps / 1e3, 3)},
        "hbm_fraction": round(b_alg * pairs_per_s / (HBM_PEAK_GBS * 1e9), 5),
        "algorithmic_bytes_per_pair": b_alg,
        "stage_ms": {k: round(x, 5) for k, x in stB.items()},
        # every FFT-path stage: its share of the pair's algorithmic bytes over its HIP-event duration
        "stage_alg_frac": {k: round(B * alg_stage_bytes(k, n, t) / (stB[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                           for k in fft_stages},
        # every input and output of the stage moved once (intermediates, sample records, and the
        # batch's one copy of the kernel spectra)
        "stage_compulsory_frac": {k: round(B * stage_bytes(k, n, batch_fft, t, spectra=1.0 / B)
                                           / (stB[k] * 1e-3) / 1e9
                                           / HBM_PEAK_GBS, 4) for k in fft_stages},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic[dom],
                     "algorithmic_bytes_per_launch": dom_alg, "launch_ms": round(stB[dom], 5),
                     "compulsory_bytes_per_launch": B * stage_bytes(dom, n, batch_fft, t, spectra=1.0 / B)},
        "counter_bytes_per_pair": round(counter_pair) if counter_pair else None,
        "counter_over_alg": round(counter_pair / b_alg, 3) if counter_pair else None,
        "kernel_per_problem": None if msB_d is None else {
            "value": round(B * 1e3 / msB_d, 1), "unit": "pairs/s", "ms_per_step": round(msB_d, 5),
            "hbm_fraction": round(b_alg * B * 1e3 / msB_d / (HBM_PEAK_GBS * 1e9), 5),
            "note": "the same pairs with a distinct kernel per problem (h varied in the sixth digit): one copy of "
                    "the kernel spectra per problem instead of one shared copy"},
        "separate_calls": {"value": round(B * 1e3 / msB_sep, 1), "unit": "pairs/s", "ms_per_step": round(msB_sep, 5),
                           "ms_per_step_runs": [round(x, 5) for x in runs_sep],
                           "note": "the same pairs as a forward call then a transpose call (a join of the "
                                   "problem ranges between them)"},
        "single_problem": {"value": round(1e3 / ms1, 1), "unit": "pairs/s", "ms_per_pair": round(ms1, 5),
                           "hbm_fraction": round(b_alg * 1e3 / ms1 / (HBM_PEAK_GBS * 1e9), 5),
                           "stage_ms": {k: round(x, 5) for k, x in st1.items()}},
    }
    del batch, c_all, s_all, g_all
    torch.cuda.empty_cache()
    if not args.no_window:
        out["window_31_direct"] = window31_line(mpik, P, r, v, c1, B, args)
    if not args.no_cosine:
        out["cosine_interp"] = cosine_line(mpik, P, r, v, c1, B, args)

    if not args.no_iter:
        out["headline_iteration"] = headline_iteration(mpik, P, r, v, c1, B)
    if not args.no_uneven:
        out["uneven_batch"] = uneven_batch(mpik, S, dev)
    if not args.no_grad:
        out["differentiation"] = differentiation(S, dev)
    if not args.no_iter:
        out["iteration_configs"] = iteration_configs(mpik, S, dev, not args.no_cpu_baseline)
    if not args.no_deconv:
        out["deconvolution"] = deconvolution(mpik, S, dev, not args.no_cpu_baseline)
    if not args.no_two_stage:
        out["two_stage"] = two_stage(mpik, S, dev, not args.no_cpu_baseline)
        out["paper_runtimes"] = paper_runtimes(mpik, S, dev)
        out["experiment2"] = experiment2_line(mpik, S, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, args.cpu_seconds)
    print(json.dumps(out))
    return 0


def window31_line(mpik, P, r, v, c1, B, args):
    """The headline shape with the kernel truncated to a 63 x 63 window on the
    direct path: one problem per launch and B per launch."""
    import torch
    n, t = P.n, P.n_samples
    plan = mpik.Plan(n, P.h, 31, r, v, conv_mode="direct")
    s1 = torch.empty((t, 2), dtype=torch.float32, device=c1.device)
    g1 = torch.empty((n, n), dtype=torch.float32, device=c1.device)

    def pair1():
        plan.forward(c1, s1)
        plan.adjoint(s1, g1)

    ms1, _, _ = graph_time(pair1, args.aux_steps, args.graph_pairs, args.warmup)
    batch = mpik.Batch([(n, P.h, 31, r, v, "direct")] * B, tune=False)
    c_all = c1.reshape(-1).repeat(B).contiguous()
    s_all = torch.empty(batch.s_offsets[-1], dtype=torch.float32, device=c1.device)
    g_all = torch.empty(batch.c_offsets[-1], dtype=torch.float32, device=c1.device)

    def pairB():
        batch.forward(c_all, s_all)
        batch.adjoint(s_all, g_all)

    msB, _, _ = graph_time(pairB, args.aux_steps, group_for(args.aux_steps), args.warmup)
    stB = stage_times(batch, g_all, s_all, max(3, args.stage_reps // 4))
    flop = 2 * 2 * 3 * (2 * 31 + 1) ** 2 * n * n      # multiply-adds of both convolutions per pair
    return {"radius": 31, "conv_path": "direct", "single_pairs_per_s": round(1e3 / ms1, 1),
            "batch": B, "batch_pairs_per_s": round(B * 1e3 / msB, 1),
            "direct_conv_tflops": round(flop * B / (msB * 1e-3) / 1e12, 2),
            "stage_ms": {k: round(x, 5) for k, x in stB.items()}}


def cosine_line(mpik, P, r, v, c1, B, args):
    """The headline workload with the cosine interpolator: the weights are
    evaluated once at plan build, so the applies run the same kernels."""
    import torch
    n, t = P.n, P.n_samples
    plan = mpik.Plan(n, P.h, P.radius, r, v, interp="cosine")
    s1 = torch.empty((t, 2), dtype=torch.float32, device=c1.device)
    g1 = torch.empty((n, n), dtype=torch.float32, device=c1.device)

    def pair1():
        plan.forward(c1, s1)
        plan.adjoint(s1, g1)

    ms1, _, _ = graph_time(pair1, args.aux_steps, args.graph_pairs, args.warmup)
    batch = mpik.Batch([(n, P.h, P.radius, r, v, "fft", "cosine")] * B, tune=False)
    c_all = c1.reshape(-1).repeat(B).contiguous()
    s_all = torch.empty(batch.s_offsets[-1], dtype=torch.float32, device=c1.device)
    g_all = torch.empty(batch.c_offsets[-1], dtype=torch.float32, device=c1.device)

    def pairB():
        batch.pair(c_all, s_all, g_all)

    msB, _, _ = graph_time(pairB, args.aux_steps, group_for(args.aux_steps), args.warmup)
    stB = stage_times(batch, g_all, s_all, max(3, args.stage_reps // 4))
    out = {"interp": "cosine", "conv_path": plan.conv_mode, "fft_size": plan.fft_size,
           "single_pairs_per_s": round(1e3 / ms1, 1), "batch": B, "batch_pairs_per_s": round(B * 1e3 / msB, 1),
           "stage_ms": {k: round(x, 5) for k, x in stB.items()}}
    del batch, c_all, s_all, g_all
    torch.cuda.empty_cache()
    return out


def deconvolution(mpik, S, dev, with_oracle, count=64, n_it=9, snr_db=30.0):
    """The Deconvolution Stage at the headline grid: `count` problems of
    256^2 with the full trace kernel (R = 255, FFT with M = 512), ZeroShot-PnP
    with ten passes, nu0 = 1e-5, CG tolerance 1e-3, 5% trimming and the
    Gaussian stand-in for the denoiser, float32.  The trace images
    u = C rho + noise (ellipse-and-line phantoms, 30 dB) are made on the
    device before the timed region.  One problem per call is timed too, and
    the float64 oracle runs the same deconvolution of one problem on the host
    (one thread) as the CPU reference."""
    import numpy as np
    import torch
    P = S.headline()
    n, R, h = P.n, 255, P.h
    tr = S.lissajous(64, ax=0.8, ay=0.8)                      # the plan's samples play no part
    r = torch.tensor(S.to_f32(tr.r), dtype=torch.float32, device=dev)
    v = torch.tensor(S.to_f32(tr.v), dtype=torch.float32, device=dev)
    kw = dict(n_it=n_it, nu0=1e-5, tol=1e-3, max_iter=10000, clip_pct=5.0, sigma_px=0.5, radius=2)

    def inputs(B):
        batch = mpik.Batch([(n, h, R, r, v, "fft")] * B, tune=False)
        rho = np.stack([S.ellipses_and_line(n, 100 + b) for b in range(B)])
        clean = batch.trace_conv(torch.tensor(rho, dtype=torch.float32, device=dev).reshape(-1))
        clean = clean.double().cpu().numpy().reshape(B, n, n)
        u = np.stack([S.add_noise(clean[b], snr_db, seed=b) for b in range(B)])
        return batch, torch.tensor(S.to_f32(u), dtype=torch.float32, device=dev).reshape(-1), rho

    def timed(batch, u, reps):
        batch.pnp(u, **kw)                                    # warm: workspace, code paths
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            out, info = batch.pnp(u, **kw)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps, out, info

    batch, u, rho = inputs(count)
    ms, out, info = timed(batch, u, 2)
    steps = np.array(info["cg_steps"])                        # [problem][pass]
    rec_err = [float(np.linalg.norm(x.double().cpu().numpy().reshape(n, n) - rho[b]) / np.linalg.norm(rho[b]))
               for b, x in enumerate(batch.c_views(out))]
    rec = {"workload": f"deconvolution_256: {count} x 256^2 trace images, R=255 (FFT, M=512), "
                       f"ZeroShot-PnP {n_it + 1} passes, nu0=1e-5, CG tol 1e-3, 5% trim, Gaussian stand-in",
           "problems": count, "grid": n, "radius": batch.info[0]["radius"], "fft_size": batch.info[0]["fft_size"],
           "passes": n_it + 1, "dtype": "f32", "ms": round(ms, 3),
           "deconvolutions_per_s": round(count * 1e3 / ms, 2),
           "cg_steps_per_problem": round(float(steps.sum(axis=1).mean()), 1),
           "cg_steps_max_pass": int(steps.max()),
           "ms_per_batched_cg_step": round(ms / float(steps.max(axis=0).sum()), 4),
           "relative_error_to_phantom": round(float(np.mean(rec_err)), 4)}
    del batch, u
    b1, u1, _ = inputs(1)
    ms1, _, info1 = timed(b1, u1, 3)
    rec["single_problem"] = {"ms": round(ms1, 3), "deconvolutions_per_s": round(1e3 / ms1, 2),
                             "cg_steps": int(np.sum(info1["cg_steps"][0]))}
    if with_oracle:
        try:
            from threadpoolctl import threadpool_limits
            limiter = threadpool_limits(1)
        except Exception:
            limiter = None
        import oracle as O
        u0 = u1.double().cpu().numpy().reshape(n, n)
        t0 = time.perf_counter()
        O.zeroshot_pnp(u0, h, R, n_it, 1e-5, tol=1e-3, max_iter=10000, clip_pct=5.0, sigma_px=0.5, radius_d=2)
        dt = time.perf_counter() - t0
        if limiter is not None:
            limiter.restore_original_limits()
        rec["oracle_deconvolutions_per_s"] = round(1.0 / dt, 4)
        rec["oracle_sample"] = "one 256^2 problem, the same ten passes, float64 numpy on one host thread"
    del b1, u1
    torch.cuda.empty_cache()
    return rec


def core_step_roofline(count, n, t, ms_per_step):
    """HBM roofline of one batched Core Stage CG step (float32 sampling,
    float64 vectors).  Compulsory bytes per problem: launch A reads r and the
    previous direction and writes the new direction and the Laplacian
    (4 x 24 N^2), reads the sample records (24 T) and writes I p (8 T);
    launch B reads I p and the records (32 T), the Laplacian and the
    direction (2 x 24 N^2), and reads and writes x and r (4 x 24 N^2):
    240 N^2 + 64 T bytes."""
    per = 240 * n * n + 64 * t
    achieved = count * per / (ms_per_step * 1e-3) / 1e9
    return {"bound": "hbm", "algorithmic_bytes_per_step": count * per, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)}


def two_stage(mpik, S, dev, with_oracle, count=64, snr_db=30.0, gamma=1e-3):
    """The paper's reconstruction from the signals: Core Stage (variational
    field reconstruction with cosine interpolation, gamma = 1e-3, CG tolerance
    1e-3), trace image, then the ZeroShot-PnP deconvolution (ten passes,
    nu0 = 1e-5, tolerance 1e-3, 5% trimming, Gaussian stand-in).  `count`
    problems of the headline shape (256^2, 53,856 Lissajous samples, full
    kernel R = 255 for the trace convolution), float32; the signals
    s = A c + noise (ellipse-and-line phantoms, 30 dB) are made on the device
    before the timed region.  The float64 oracle's Core Stage step rate is
    measured on a bounded sample of steps of one problem."""
    import numpy as np
    import torch
    P = S.headline()
    n, R, t = P.n, 255, P.n_samples
    r = torch.tensor(S.to_f32(P.traj.r), dtype=torch.float32, device=dev)
    v = torch.tensor(S.to_f32(P.traj.v), dtype=torch.float32, device=dev)
    batch = mpik.Batch([(n, P.h, R, r, v, "fft", "cosine")] * count, tune=False)
    c = np.stack([S.ellipses_and_line(n, 200 + b) for b in range(count)])
    clean = batch.forward(torch.tensor(c, dtype=torch.float32, device=dev).reshape(-1))
    clean = clean.double().cpu().numpy().reshape(count, t, 2)
    s_all = torch.tensor(S.to_f32(np.stack([S.add_noise(clean[b], snr_db, seed=b) for b in range(count)])),
                         dtype=torch.float32, device=dev).reshape(-1)
    pnp_kw = dict(n_it=9, nu0=1e-5, tol=1e-3, max_iter=10000, clip_pct=5.0, sigma_px=0.5, radius=2)

    def run():
        field, steps = batch.core_stage(s_all, gamma=gamma, tol=1e-3, max_iter=10000)
        u = batch.field_trace(field)
        rho, info = batch.pnp(u, **pnp_kw)
        return field, steps, rho, info

    run()                                                     # warm: workspaces, graphs
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    field, steps = batch.core_stage(s_all, gamma=gamma, tol=1e-3, max_iter=10000)
    ev[1].record()
    rho, info = batch.pnp(batch.field_trace(field), **pnp_kw)
    ev[2].record()
    torch.cuda.synchronize()
    core_ms, pnp_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    rho_h = rho.double().cpu().numpy().reshape(count, n, n)
    err = float(np.mean([np.linalg.norm(rho_h[b] - c[b]) / np.linalg.norm(c[b]) for b in range(count)]))
    rec = {"workload": f"two_stage_256: {count} x (256^2 grid, 53,856 samples, cosine interpolation) Core Stage "
                       f"gamma={gamma:g} tol 1e-3, trace, ZeroShot-PnP 10 passes (R=255 FFT)",
           "problems": count, "dtype": "f32", "ms": round(core_ms + pnp_ms, 3),
           "reconstructions_per_s": round(count * 1e3 / (core_ms + pnp_ms), 2),
           "core_stage_ms": round(core_ms, 3), "core_cg_steps_max": int(max(steps)),
           "ms_per_batched_core_step": round(core_ms / max(1, max(steps)), 4),
           "core_step_roofline": core_step_roofline(count, n, t, core_ms / max(1, max(steps))),
           "deconvolution_ms": round(pnp_ms, 3),
           "relative_error_to_phantom": round(err, 4)}
    if with_oracle:
        try:
            from threadpoolctl import threadpool_limits
            limiter = threadpool_limits(1)
        except Exception:
            limiter = None
        import oracle as O
        rr, vv = S.to_f32(P.traj.r), S.to_f32(P.traj.v)
        s0 = s_all[:2 * t].double().cpu().numpy().reshape(t, 2)
        b0 = O.core_rhs(s0, rr, vv, n)
        k = 40
        t0 = time.perf_counter()
        O.cg(lambda a: O.core_normal(a, rr, vv, gamma), b0, 0.0, k)
        dt = time.perf_counter() - t0
        if limiter is not None:
            limiter.restore_original_limits()
        rec["oracle_core_steps_per_s"] = round(k / dt, 2)
        rec["oracle_sample"] = f"{k} Core Stage CG steps of one 256^2 problem, float64 numpy, one host thread"
    del batch, s_all, field, rho
    torch.cuda.empty_cache()
    return rec


def experiment2_line(mpik, S, dev, count=64, n=128, keep=100, snr_db=30.0, gamma=1e-3):
    """The Experiment-2 inputs on 64 problems: the drive-plus-excitation
    figure at 2,000,000 full-rate samples, velocities by forward differences
    on the device, one sample in 100 kept (20,000), the anisotropic gradient
    G = diag(1.39, -3.16) (velocity -G dr/dt), the x receive channel alone,
    128^2 grids with the full kernel (FFT), cosine interpolation, float32.
    Phantoms: two bars with gaps from 0.04 to 0.3, and blobs.  Timed: Core
    Stage (gamma = 1e-3, tolerance 1e-3), the trace (A_xx), ZeroShot-PnP with
    K_xx (ten passes, nu0 = 4e-2, tolerance 1e-3).  The signals s = A c +
    noise (30 dB) are made on the device beforehand."""
    import numpy as np
    import torch
    grad = (1.39, -3.16)
    full = S.experiment2(2_000_000)
    dt = full.t[1] - full.t[0]
    r_full = torch.tensor(S.to_f32(full.r), dtype=torch.float32, device=dev)
    mpik.velocity_forward_difference(r_full, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v_fd = mpik.velocity_forward_difference(r_full, dt)
    torch.cuda.synchronize()
    fd_ms = (time.perf_counter() - t0) * 1e3
    r = r_full[::keep].contiguous()
    v = (-(v_fd[::keep] * torch.tensor(grad, dtype=torch.float32, device=dev))).contiguous()
    h = S.h_fwhm2(n)
    batch = mpik.Batch([(n, h, n - 1, r, v, "fft", "cosine")] * count, tune=False, channels="x", grad=grad)
    c = np.stack([S.bars(n, 0.04 + 0.26 * b / (count - 1)) if b % 2 == 0 else S.blobs(n, 500 + b)
                  for b in range(count)])
    clean = batch.forward(torch.tensor(c, dtype=torch.float32, device=dev).reshape(-1))
    clean = clean.double().cpu().numpy().reshape(count, -1, 2)
    s_all = torch.tensor(S.to_f32(np.stack([S.add_noise(clean[b], snr_db, seed=b) for b in range(count)])),
                         dtype=torch.float32, device=dev).reshape(-1)
    pnp_kw = dict(n_it=9, nu0=4e-2, tol=1e-3, max_iter=10000, clip_pct=5.0, sigma_px=0.5, radius=2)

    def run():
        field, steps = batch.core_stage(s_all, gamma=gamma, tol=1e-3, max_iter=10000)
        rho, info = batch.pnp(batch.field_trace(field), **pnp_kw)
        return steps, rho

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, rho = run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    rho_h = rho.double().cpu().numpy().reshape(count, n, n)
    err = float(np.mean([np.linalg.norm(rho_h[b] - c[b]) / np.linalg.norm(c[b]) for b in range(count)]))
    out = {"workload": f"experiment2_{n}: {count} x ({n}^2 grid, 2,000,000 samples thinned 1:{keep}, "
                       "G = diag(1.39, -3.16), x channel, cosine) Core Stage + K_xx ZeroShot-PnP",
           "problems": count, "samples_kept": int(r.shape[0]), "dtype": "f32", "ms": round(ms, 3),
           "reconstructions_per_s": round(count * 1e3 / ms, 2), "core_cg_steps_max": int(max(steps)),
           "velocity_forward_difference_ms": round(fd_ms, 4), "relative_error_to_phantom": round(err, 4),
           "note": "host wall clock around one warm batched reconstruction, synchronised"}
    del batch, s_all, rho
    torch.cuda.empty_cache()
    return out


# The paper's only timings (its runtime table): the whole reconstruction (Core
# Stage and ZeroShot-PnP) on the EMWA data, one 1632-sample Lissajous period,
# on an Intel i9-13900KS and an NVIDIA RTX A6000 (precision not stated).
PAPER_RUNTIMES_S = {21: {"cpu": 0.46, "gpu": 1.56}, 100: {"cpu": 5.84, "gpu": 3.36}}
PAPER_HARDWARE = "Intel i9-13900KS (CPU), NVIDIA RTX A6000 (GPU), Windows 11"


def paper_runtimes(mpik, S, dev, snr_db=30.0, gamma=1e-3):
    """The workload shape of the paper's runtime table, on synthetic data: one
    problem on the 21 x 21 and 100 x 100 grids, 1632 samples of one period of
    the 17:16 Lissajous figure, cosine interpolation, the full kernel (FFT),
    float32; Core Stage (gamma = 1e-3, CG tolerance 1e-3), trace image,
    ZeroShot-PnP (ten passes, nu0 = 1e-5, tolerance 1e-3, 5 % trimming,
    Gaussian stand-in).  The signal s = A c + noise (ellipse-and-line phantom,
    30 dB) is made before the timed region; each reconstruction is timed
    once warm.  The paper's figures are quoted beside it for context: other
    hardware, the measured EMWA data, and its learned denoiser."""
    import numpy as np
    import torch
    out = {}
    for n in (21, 100):
        tr = S.lissajous(S.SAMPLES_PER_PERIOD, ax=0.95, ay=0.95)
        r = torch.tensor(S.to_f32(tr.r), dtype=torch.float32, device=dev)
        v = torch.tensor(S.to_f32(tr.v), dtype=torch.float32, device=dev)
        batch = mpik.Batch([(n, S.h_fwhm2(n), n - 1, r, v, "fft", "cosine")], tune=False)
        c = S.ellipses_and_line(n, 7)
        clean = batch.forward(torch.tensor(S.to_f32(c), dtype=torch.float32, device=dev).reshape(-1))
        s_all = torch.tensor(S.to_f32(S.add_noise(clean.double().cpu().numpy().reshape(-1, 2), snr_db, seed=n)),
                             dtype=torch.float32, device=dev).reshape(-1)

        def run():
            field, steps = batch.core_stage(s_all, gamma=gamma, tol=1e-3, max_iter=10000)
            rho, info = batch.pnp(batch.field_trace(field), n_it=9, nu0=1e-5, tol=1e-3, max_iter=10000,
                                  clip_pct=5.0, sigma_px=0.5, radius=2)
            return steps, rho, info

        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, rho, info = run()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        err = float(np.linalg.norm(rho.double().cpu().numpy().reshape(n, n) - c) / np.linalg.norm(c))
        out[f"grid_{n}"] = {"samples": S.SAMPLES_PER_PERIOD, "ms": round(ms, 3), "core_cg_steps": int(steps[0]),
                            "pnp_cg_steps": int(sum(info["cg_steps"][0])),
                            "relative_error_to_phantom": round(err, 4),
                            "paper_s": PAPER_RUNTIMES_S[n]}
        del batch
    out["paper_hardware"] = PAPER_HARDWARE
    out["note"] = "host wall clock around one warm reconstruction, synchronised; context only, not a target"
    torch.cuda.empty_cache()
    return out


def iteration_configs(mpik, S, dev, with_oracle, oracle_seconds=3.0):
    """Iterations per second of the plain solves: 32^2 / R = 7 / float64 /
    50 Landweber steps; 128^2 / R = 31 / 200 denoised steps; 256^2 / full
    kernel / 2^17 samples of the perturbed partial trajectory / 200 denoised
    steps.  The float64 oracle's iteration rate on the host (one thread, a few
    steps) is reported beside each."""
    import numpy as np
    import torch
    out = {}
    for P in (S.plain_f64(), S.plain_f32(), S.independence()):
        dt = torch.float64 if P.dtype == "f64" else torch.float32
        tt = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), dtype=dt, device=dev).contiguous()
        plan = mpik.Plan(P.n, P.h, P.radius, tt(P.traj.r), tt(P.traj.v))
        s = plan.forward(tt(P.c))
        x = torch.randn((P.n, P.n), dtype=dt, device=dev)
        for _ in range(10):
            x = plan.adjoint(plan.forward(x / x.norm()))
        tau = 0.9 / float(x.norm())
        sigma = 0.5 if P.denoise else 0.0
        c = torch.zeros((P.n, P.n), dtype=dt, device=dev)
        plan.iterate(s, c, P.n_iter, tau, sigma, 2)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(3):
            plan.iterate(s, c, P.n_iter, tau, sigma, 2)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 3
        rec = {"grid": P.n, "samples": P.n_samples, "radius": plan.radius, "conv_path": plan.conv_mode,
               "dtype": "f64" if dt == torch.float64 else "f32", "iterations": P.n_iter,
               "denoise": bool(P.denoise), "solve_ms": round(ms, 3),
               "iterations_per_s": round(P.n_iter * 1e3 / ms, 1)}
        if with_oracle:
            rec["oracle_iterations_per_s"] = oracle_iteration_rate(P, tau, oracle_seconds)
        out[P.name] = rec
        del plan
    return out


def oracle_iteration_rate(P, tau, budget_s):
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:
        limiter = None
    import numpy as np
    import oracle as O
    from paper_2505_22797_amd import synth as S
    rnd = (lambda a: a) if P.dtype == "f64" else S.to_f32
    model = O.Model(P.n, P.h, P.radius, rnd(P.traj.r), rnd(P.traj.v))
    s = model.forward(rnd(P.c))
    c = np.zeros((P.n, P.n))
    steps = 0
    t0 = time.perf_counter()
    while True:
        c = O.iterate(model, s, c, tau, 1, sigma_px=0.5 if P.denoise else None, radius=2)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 200:
            break
    del limiter
    return round(steps / el, 3)


def profile_batch(mpik, P, r, v, c1, B, steps):
    """Run for hardware counters: one batched pair, then every kernel stage
    launched `steps` times over the whole batch (the launches whose durations
    give the roofline), and one plain device copy of 256 MiB, whose FETCH_SIZE
    and WRITE_SIZE calibrate the counters against a known byte count."""
    import torch
    n, t = P.n, P.n_samples
    batch = mpik.Batch([(n, P.h, P.radius, r, v, "fft")] * B, tune=False)
    c_all = c1.reshape(-1).repeat(B).contiguous()
    s_all = torch.empty(batch.s_offsets[-1], dtype=torch.float32, device=c1.device)
    g_all = torch.empty(batch.c_offsets[-1], dtype=torch.float32, device=c1.device)
    batch.pair(c_all, s_all, g_all)
    for k in range(len(batch.stages())):
        batch.launch_stage(k, max(1, min(steps, 20)), g_all, s_all)
    src = torch.ones(64 << 20, dtype=torch.float32, device=c1.device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile_batch": B, "copy_bytes": src.numel() * 4, "grid": n, "samples": t}))
    return 0


def headline_iteration(mpik, P, r, v, c1, B, n_iter=50):
    """The hot loop itself at the headline shape: B problems, n_iter
    denoised iterations c <- D(c - tau A^T (A c - s)) through the library's
    batched iteration (one captured graph per iteration, each problem range's
    transpose right after its forward, the gradient step fused into the last
    transpose stage).  Reported as A + A^T pairs per second."""
    import torch
    n, t = P.n, P.n_samples
    batch = mpik.Batch([(n, P.h, P.radius, r, v, "fft")] * B, tune=False)
    c_all = torch.zeros(batch.c_offsets[-1], dtype=torch.float32, device=c1.device)
    s_all = batch.forward(c1.reshape(-1).repeat(B).contiguous())
    taus = [1e-4] * B
    batch.iterate(s_all, c_all, n_iter, taus, 0.5, 2)     # warm: captures the iteration graphs
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    batch.iterate(s_all, c_all, n_iter, taus, 0.5, 2)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    del batch, c_all, s_all
    torch.cuda.empty_cache()
    return {"problems": B, "iterations": n_iter, "ms": round(ms, 3), "ms_per_iteration": round(ms / n_iter, 5),
            "pairs_per_s": round(B * n_iter * 1e3 / ms, 1), "denoise": "Gaussian sigma 0.5 px, radius 2"}


def uneven_batch(mpik, S, dev, n_iter=50):
    """64 uneven problems (N in {64..256}, 10k-120k samples, three trajectory
    kinds, h within +-20%, R = 31), 50 denoised iterations: one batched
    graph-replayed solve against 64 sequential single-problem solves."""
    import torch
    probs = S.batch_problems(64)
    tt = lambda a: torch.tensor(S.to_f32(a), dtype=torch.float32, device=dev)
    specs = [(p.n, p.h, p.radius, tt(p.traj.r), tt(p.traj.v)) for p in probs]
    t0 = time.perf_counter()
    batch = mpik.Batch(specs, tune=True)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    c_all = torch.zeros(batch.c_offsets[-1], dtype=torch.float32, device=dev)
    s_all = torch.randn(batch.s_offsets[-1], dtype=torch.float32, device=dev)
    taus = [1e-4] * len(probs)
    batch.iterate(s_all, c_all, n_iter, taus, 0.5, 2)     # warm: captures the iteration graphs
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    batch.iterate(s_all, c_all, n_iter, taus, 0.5, 2)
    b.record()
    torch.cuda.synchronize()
    ms_batched = a.elapsed_time(b)
    modes = {}
    for inf in batch.info:
        key = inf["conv_mode"] + (f"/s{inf['slices']}" if inf["conv_mode"] == "direct" else "")
        modes[key] = modes.get(key, 0) + 1
    del batch
    plans = [mpik.Plan(*sp) for sp in specs]
    cs = [torch.zeros((p.n, p.n), dtype=torch.float32, device=dev) for p in plans]
    ss = [torch.randn((p.n_samples, 2), dtype=torch.float32, device=dev) for p in plans]
    for p, c, s in zip(plans, cs, ss):
        p.iterate(s, c, n_iter, 1e-4, 0.5, 2)     # warm: captures the iteration graphs
    torch.cuda.synchronize()
    a.record()
    for p, c, s in zip(plans, cs, ss):
        p.iterate(s, c, n_iter, 1e-4, 0.5, 2)
    b.record()
    torch.cuda.synchronize()
    ms_seq = a.elapsed_time(b)
    return {"problems": len(probs), "iterations": n_iter, "batched_ms": round(ms_batched, 3),
            "sequential_ms": round(ms_seq, 3), "speedup": round(ms_seq / ms_batched, 3),
            "batched_iterations_per_s": round(len(probs) * n_iter * 1e3 / ms_batched, 1),
            "build_and_tune_s": round(build_s, 3), "paths": modes}


def differentiation(S, dev, reps=3):
    """8 problems at 256^2, 53,856 samples, R = 31: the unrolled K = 20
    denoised solve with checkpoints every 5, forward and hand-written backward
    (gradients for c0, h and the two trajectory amplitudes), against the plain
    K = 20 solve at the same shape, plus the rebuild of the plan with the
    dK/dh tables that every change of h or of the trajectory needs."""
    import torch
    from paper_2505_22797_amd import autograd as AG
    probs = S.gradient_problems(8)
    B, n, R, T = len(probs), probs[0].n, probs[0].radius, probs[0].n_samples
    shape = S.lissajous(T, ax=1.0, ay=1.0)
    rho = torch.tensor(S.to_f32(shape.r), dtype=torch.float32, device=dev)
    nu = torch.tensor(S.to_f32(shape.v), dtype=torch.float32, device=dev)
    op = AG.TrajectoryOperator([n] * B, [R] * B, [rho] * B, [nu] * B)
    h = torch.tensor([p.h * 1.05 for p in probs], dtype=torch.float64)
    amp = torch.full((B,), S.AMPLITUDE * 0.98, dtype=torch.float64)
    truth = torch.cat([torch.tensor(S.to_f32(p.c), dtype=torch.float32, device=dev).reshape(-1) for p in probs])
    plan = op.plan(h, amp, amp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()        # rebuilds at new parameter values, as after an optimiser step
    for i in range(3):
        op.plan(h * (1.0 + 1e-4 * (i + 1)), amp, amp)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3 / 3
    s_all = plan.forward(truth)
    x = torch.randn_like(truth)          # step 0.9 / lambda_max from a short power iteration
    for _ in range(10):
        x = plan.adjoint(plan.forward(x / x.norm()))
    taus = [0.9 / float(x.norm())] * B
    K, every, sigma = 20, 5, 0.5

    def grad_step():
        c0 = torch.zeros_like(truth, requires_grad=True)
        hh, ax, ay = (t.clone().requires_grad_(True) for t in (h, amp, amp))
        c = AG.unrolled_solve(op, s_all, c0, hh, ax, ay, taus, n_iter=K, sigma_px=sigma, radius=2, every=every)
        loss = torch.sum((c - truth) ** 2)
        return torch.autograd.grad(loss, (c0, hh, ax, ay))

    grad_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        grad_step()
    torch.cuda.synchronize()
    grad_ms = (time.perf_counter() - t0) * 1e3 / reps
    c = torch.zeros_like(truth)
    plan.iterate(s_all, c, K, taus, sigma, 2)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        plan.iterate(s_all, c, K, taus, sigma, 2)
    b.record()
    torch.cuda.synchronize()
    plain_ms = a.elapsed_time(b) / reps
    return {"problems": B, "grid": n, "samples": T, "radius": R, "iterations": K, "checkpoint_every": every,
            "forward_backward_ms": round(grad_ms, 3), "plain_solve_ms": round(plain_ms, 3),
            "ratio": round(grad_ms / plain_ms, 2), "plan_rebuild_ms": round(build_ms, 3),
            "gradient_steps_per_s": round(1e3 / (grad_ms + build_ms), 2)}


def cpu_baseline(P, budget_s: float) -> dict:
    """The float64 oracle pair on the host (numpy FFT convolution, bincount
    transpose), single-threaded, on a bounded number of pairs."""
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:
        limiter = None
    import oracle as O
    from paper_2505_22797_amd import synth as S
    r, v, c = S.to_f32(P.traj.r), S.to_f32(P.traj.v), S.to_f32(P.c)
    model = O.Model(P.n, P.h, P.radius, r, v)
    pairs = 0
    t0 = time.perf_counter()
    while True:
        model.adjoint(model.forward(c))
        pairs += 1
        el = time.perf_counter() - t0
        if el >= budget_s or pairs >= 400:
            break
    del limiter
    import numpy
    import scipy
    return {"value": round(pairs / el, 4), "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"{pairs} A+A^T pairs of the 256^2 / 53,856-sample / R=255 operator in float64 numpy "
                      f"(FFT convolution, bincount transpose), {el:.1f} s, one thread of "
                      f"{os.cpu_count()} visible cores",
            "cpu_model": cpu_model(), "numpy": numpy.__version__, "scipy": scipy.__version__}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    sys.exit(main())
