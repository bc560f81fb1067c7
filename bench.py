#!/usr/bin/env python3
"""Throughput of the MPI model operator pair A + A^T on one MI355X.

Workload: 256 x 256 grid, 53,856 Lissajous samples (33 periods of 1632,
17:16 cycles), full-size Langevin kernel (R = 255, FFT path with M = 512),
float32, the ellipse-and-line phantom.  One step is one A + A^T pair
(s = A c, then c' = A^T s), all inputs resident in device memory.  The timed
steps are replayed from a captured HIP graph of `--graph-pairs` pairs.

Also reported: per-kernel durations from HIP events on the launch stream
(each stage launched alone through the library's diagnostic entry point),
the roofline of the dominant kernel, the pair's fraction of HBM peak for the
algorithmic bytes 56 N^2 + 48 T, and the float64 CPU oracle timed on a
bounded sample of pairs on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
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


def stage_bytes(name: str, n: int, m: int, t: int, elem: int = 4) -> float:
    """Compulsory bytes of one launch of a stage: each input and output moved
    once (intermediate spectra included, plan constants included)."""
    hh = m // 2 + 1
    cplx = 2 * elem
    samp = t * (4 * elem + 4 + 4)          # (fx, fy, vx, vy), base cell, permutation
    return {
        "fwd_rows": elem * n * n + cplx * hh * n,
        "fwd_cols": cplx * hh * n + elem * 3 * hh * hh + 3 * cplx * n * hh,
        "fwd_rows_gather": 3 * cplx * n * hh + samp + 2 * elem * t,
        "adj_scatter_rows": 4 * (4 * t + n * n) + samp + 2 * elem * t + 3 * cplx * hh * n,
        "adj_cols": 3 * cplx * hh * n + elem * 3 * hh * hh + cplx * n * hh,
        "adj_rows": cplx * n * hh + elem * n * n,
    }[name]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--graph-pairs", type=int, default=20)
    ap.add_argument("--stage-reps", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the operator runs on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    sys.path.insert(0, HERE)
    from paper_2505_22797_amd import mpik
    from paper_2505_22797_amd import synth as S

    P = S.headline()
    n, t = P.n, P.n_samples
    dev = torch.device("cuda:0")
    r = torch.tensor(S.to_f32(P.traj.r), dtype=torch.float32, device=dev)
    v = torch.tensor(S.to_f32(P.traj.v), dtype=torch.float32, device=dev)
    plan = mpik.Plan(n, P.h, P.radius, r, v)
    c = torch.tensor(P.c, dtype=torch.float32, device=dev)
    s = torch.empty((t, 2), dtype=torch.float32, device=dev)
    c2 = torch.empty((n, n), dtype=torch.float32, device=dev)

    def pair():
        plan.forward(c, s)
        plan.adjoint(s, c2)

    # warm-up, eager
    for _ in range(args.warmup):
        pair()
    torch.cuda.synchronize()

    # eager timing (host launch path included)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_eager = max(20, args.steps // 4)
    e0.record()
    for _ in range(n_eager):
        pair()
    e1.record()
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / n_eager

    # graph of G pairs, replayed for the timed steps
    G = max(1, args.graph_pairs)
    K = max(G, (args.steps + G - 1) // G * G)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pair()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(G):
            pair()
    for _ in range(2):
        graph.replay()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record()
    for _ in range(K // G):
        graph.replay()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = t0.elapsed_time(t1) / K
    pairs_per_s = 1e3 / ms_per_step

    # per-stage kernel durations (HIP events on the launch stream)
    stages = plan.stages()
    stage_ms = {}
    pair()
    torch.cuda.synchronize()
    for k, name in enumerate(stages):
        plan.launch_stage(k, 3, c2, s)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        plan.launch_stage(k, args.stage_reps, c2, s)
        b.record()
        torch.cuda.synchronize()
        stage_ms[name] = a.elapsed_time(b) / args.stage_reps
    dom = max(stage_ms, key=stage_ms.get)
    dom_bytes = stage_bytes(dom, n, plan.fft_size, t) if plan.conv_mode == "fft" else None
    achieved = dom_bytes / (stage_ms[dom] * 1e-3) / 1e9 if dom_bytes else None

    traffic = None
    pmc = os.path.join(HERE, "profiles", f"{dom}_headline_256_pmc.json")
    if os.path.exists(pmc):
        rec = json.load(open(pmc))
        if rec.get("src_digest") == src_digest():
            traffic = rec.get("hbm_bytes_per_launch")

    b_alg = 56 * n * n + 48 * t
    out = {
        "metric": "A+A^T applies/s at 256^2 grid, 53,856 samples (fraction of HBM peak)",
        "value": round(pairs_per_s, 1),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "headline_256: N=256, T=53856 Lissajous 17:16, R=255 (FFT, M=512), one problem",
                   "grid": n, "samples": t, "radius": plan.radius, "fft_size": plan.fft_size,
                   "conv_path": plan.conv_mode, "graph_pairs": G},
        "hbm_fraction": round(b_alg * pairs_per_s / (HBM_PEAK_GBS * 1e9), 5),
        "algorithmic_bytes_per_pair": b_alg,
        "eager_ms_per_pair": round(eager_ms, 5),
        "wall_s": round(wall, 4),
        "stage_ms": {k: round(x, 5) for k, x in stage_ms.items()},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 2) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5) if achieved else None,
                     "traffic": traffic, "algorithmic_bytes_per_launch": dom_bytes},
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, args.cpu_seconds)
    print(json.dumps(out))
    return 0


def cpu_baseline(P, budget_s: float) -> dict:
    """The float64 oracle pair on the host: FFT convolution through numpy,
    bincount transpose; single-threaded."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(1)
    except Exception:
        limit = None
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
        if el >= budget_s or pairs >= 200:
            break
    if limit is not None:
        limit.unregister() if hasattr(limit, "unregister") else None
    return {"value": round(pairs / el, 4), "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"{pairs} A+A^T pairs of the 256^2 / 53,856-sample / R=255 operator, float64 numpy "
                      f"(FFT convolution, bincount transpose), {el:.1f} s on {os.cpu_count()} visible cores"}


if __name__ == "__main__":
    sys.exit(main())
