"""GPU parity at the configurations the benchmark measures, call for call.

* The headline pair call: B problems of the 256^2 / 53,856-sample shape with
  the full-size kernel (R = 255, FFT with M = 512), built as the benchmark
  builds them (no tuning, the default column-kernel shape and problem-range
  split), through the one-call pair entry (s = A c, then A^T s).  B = 64 runs
  as two problem ranges on side streams, B = 32 and 16 as four.  Every
  problem has its own concentration, so a range that read or wrote another
  range's problem would fail; the benchmark's own inputs (one concentration
  repeated) are checked as well.
* The trajectory-independence workload at its full 200 denoised iterations.
* The uneven 64-problem batch solved in one tuned batched call of 50
  denoised iterations, compared problem by problem with the oracle on a
  subset that covers every grid size and every trajectory kind.

Besides the relative L2 error of the whole array (the parity metric), every
comparison bounds the element-wise error max |got - ref| / max |ref|, so that
an error confined to a few cells or samples (hull cells, a heavy bin, a range
edge) cannot hide in the norm.  Operator: eq. (coreoperator) sampled and
contracted per eq. (core:formula); iteration c <- D(c - tau A^T (A c - s)).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2505_22797_amd import mpik
from paper_2505_22797_amd import synth as S
from gpu_helpers import dev, max_rel, rel_l2, rounded

pytestmark = pytest.mark.gpu

F32_APPLY = 1e-5
F32_ITER = 1e-4


def _headline_batch(B):
    """The benchmark's batch: B copies of the headline problem description."""
    P = S.headline()
    r, v = S.to_f32(P.traj.r), S.to_f32(P.traj.v)
    batch = mpik.Batch([(P.n, P.h, P.radius, dev(r, torch.float32), dev(v, torch.float32), "fft")] * B,
                       tune=False)
    return P, r, v, batch


@pytest.fixture(scope="module")
def headline_refs():
    """Oracle pairs (s = A c, g = A^T s) for 64 distinct phantoms at the
    headline shape, plus the benchmark's own phantom."""
    P = S.headline()
    r, v = S.to_f32(P.traj.r), S.to_f32(P.traj.v)
    model = O.Model(P.n, P.h, P.radius, r, v)
    cs = [rounded(S.ellipses_and_line(P.n, 5000 + b), torch.float32) for b in range(64)]
    refs = []
    for c in cs:
        s = model.forward(c)
        refs.append((s, model.adjoint(rounded(s, torch.float32))))
    c_bench = S.to_f32(P.c)
    s_b = model.forward(c_bench)
    return model, cs, refs, (c_bench, s_b, model.adjoint(rounded(s_b, torch.float32)))


@pytest.mark.parametrize("B", [64, 32, 16])
def test_headline_pair_call_every_problem(headline_refs, B):
    """The timed call itself: B distinct problems through the pair entry,
    every problem's s and A^T s against the oracle.  The transpose is
    compared with the oracle's A^T of the float32 forward result the pair
    call fed it (the call's own s)."""
    model, cs, refs, _ = headline_refs
    P, r, v, batch = _headline_batch(B)
    assert all(i["conv_mode"] == "fft" and i["fft_size"] == 512 and i["radius"] == 255 for i in batch.info)
    c_all = torch.cat([dev(cs[b], torch.float32).reshape(-1) for b in range(B)])
    s_all, g_all = batch.pair(c_all)
    torch.cuda.synchronize()
    sv, gv = batch.s_views(s_all), batch.c_views(g_all)
    worst = [0.0, 0.0, 0.0, 0.0]
    for b in range(B):
        s_ref, _ = refs[b]
        s_got = sv[b].double().cpu().numpy()
        g_got = gv[b].double().cpu().numpy()
        g_ref = model.adjoint(rounded(s_got, torch.float32))
        e = (rel_l2(s_got, s_ref), max_rel(s_got, s_ref), rel_l2(g_got, g_ref), max_rel(g_got, g_ref))
        worst = [max(a, x) for a, x in zip(worst, e)]
        assert e[0] <= F32_APPLY and e[1] <= F32_APPLY, (b, e)
        assert e[2] <= F32_APPLY and e[3] <= F32_APPLY, (b, e)
    print(f"B={B}: worst forward rel-L2 {worst[0]:.2e} max-rel {worst[1]:.2e}, "
          f"transpose rel-L2 {worst[2]:.2e} max-rel {worst[3]:.2e}")


def test_headline_pair_call_bench_inputs(headline_refs):
    """The benchmark's exact inputs: 64 copies of its phantom through the
    pair entry; all 64 results against one oracle pair, and every problem
    bitwise equal to the first (the same problem in another range)."""
    model, _, _, (c_bench, s_ref, g_ref) = headline_refs
    P, r, v, batch = _headline_batch(64)
    c_all = dev(c_bench, torch.float32).reshape(-1).repeat(64).contiguous()
    s_all, g_all = batch.pair(c_all)
    torch.cuda.synchronize()
    sv, gv = batch.s_views(s_all), batch.c_views(g_all)
    s0, g0 = sv[0].double().cpu().numpy(), gv[0].double().cpu().numpy()
    g_ref = model.adjoint(rounded(s0, torch.float32))
    assert rel_l2(s0, s_ref) <= F32_APPLY and max_rel(s0, s_ref) <= F32_APPLY
    assert rel_l2(g0, g_ref) <= F32_APPLY and max_rel(g0, g_ref) <= F32_APPLY
    for b in range(1, 64):
        assert torch.equal(sv[b], sv[0]) and torch.equal(gv[b], gv[0]), b


def test_headline_separate_calls_element_wise(headline_refs):
    """The same batch as a forward call then a transpose call (the second
    figure the benchmark reports): bitwise the pair call's results."""
    _, cs, _, _ = headline_refs
    P, r, v, batch = _headline_batch(64)
    c_all = torch.cat([dev(c, torch.float32).reshape(-1) for c in cs])
    s_p, g_p = batch.pair(c_all)
    s_all = batch.forward(c_all)
    g_all = batch.adjoint(s_all)
    torch.cuda.synchronize()
    assert torch.equal(s_p, s_all) and torch.equal(g_p, g_all)


def test_independence_full_200_iterations():
    """The trajectory-independence workload: 256^2, the perturbed partial
    trajectory with 2^17 samples, full-size kernel, 20 dB noise, all 200
    denoised iterations with tau = 1/lambda_max from 100 float64 power
    iterations, against the oracle at 1e-4."""
    P = S.independence()
    r, v, c = S.to_f32(P.traj.r), S.to_f32(P.traj.v), S.to_f32(P.c)
    model = O.Model(P.n, P.h, P.radius, r, v)
    s = S.to_f32(S.add_noise(model.forward(c), P.snr_db, seed=1))
    tau = 1.0 / O.power_lambda_max(model, iters=100)
    ref = O.iterate(model, s, np.zeros((P.n, P.n)), tau, P.n_iter, sigma_px=0.5, radius=2)
    plan = mpik.Plan(P.n, P.h, P.radius, dev(r, torch.float32), dev(v, torch.float32))
    assert plan.conv_mode == "fft" and plan.fft_size == 512
    got = torch.zeros((P.n, P.n), dtype=torch.float32, device="cuda")
    plan.iterate(dev(s, torch.float32), got, P.n_iter, tau, denoise_sigma_px=0.5, denoise_radius=2)
    torch.cuda.synchronize()
    got = got.double().cpu().numpy()
    e, m = rel_l2(got, ref), max_rel(got, ref)
    print(f"independence 200 iterations: rel-L2 {e:.2e} max-rel {m:.2e}")
    assert e <= F32_ITER and m <= F32_ITER


def _uneven_subset(probs):
    """Indices covering every grid size twice and every trajectory kind
    (b mod 3) at least three times: for each size, its first problem of
    kind (size index) mod 3 and of kind (size index + 1) mod 3."""
    sizes = sorted({p.n for p in probs})
    pick = []
    for si, n in enumerate(sizes):
        for kind in (si % 3, (si + 1) % 3):
            b = next(b for b, p in enumerate(probs) if p.n == n and b % 3 == kind)
            pick.append(b)
    return pick


def test_uneven_batch_50_iterations():
    """The uneven 64-problem batch (N in {64,...,256}, 10k-120k samples,
    Lissajous / perturbed / partial, h within +-20%, R = 31) in one tuned
    batched solve of 50 denoised iterations; measured signals with 20 dB
    noise and a per-problem step 0.9/lambda_max.  Ten problems covering every
    grid size and trajectory kind are compared with the oracle at 1e-4."""
    probs = S.batch_problems(64)
    r32 = [S.to_f32(p.traj.r) for p in probs]
    v32 = [S.to_f32(p.traj.v) for p in probs]
    batch = mpik.Batch([(p.n, p.h, p.radius, dev(r32[b], torch.float32), dev(v32[b], torch.float32))
                        for b, p in enumerate(probs)], tune=True)
    pick = _uneven_subset(probs)
    assert {probs[b].n for b in pick} == {64, 96, 128, 192, 256} and {b % 3 for b in pick} == {0, 1, 2}
    s_list, taus, models = [], [], {}
    for b, p in enumerate(probs):
        if b in pick:
            M = O.Model(p.n, p.h, p.radius, r32[b], v32[b])
            models[b] = M
            s_list.append(S.to_f32(S.add_noise(M.forward(S.to_f32(p.c)), 20.0, seed=1)))
            taus.append(0.9 / O.power_lambda_max(M, iters=15))
        else:   # run in the batch, not compared: any signal, a small step
            s_list.append(S.to_f32(np.random.default_rng(b).standard_normal((p.n_samples, 2))))
            taus.append(1e-4)
    s_all = torch.cat([dev(s, torch.float32).reshape(-1) for s in s_list])
    c_all = torch.zeros(batch.c_offsets[-1], dtype=torch.float32, device="cuda")
    batch.iterate(s_all, c_all, 50, taus, denoise_sigma_px=0.5, denoise_radius=2)
    torch.cuda.synchronize()
    cv = batch.c_views(c_all)
    paths = {batch.info[b]["conv_mode"] for b in pick}
    for b in pick:
        p = probs[b]
        ref = O.iterate(models[b], s_list[b], np.zeros((p.n, p.n)), taus[b], 50, sigma_px=0.5, radius=2)
        got = cv[b].double().cpu().numpy()
        e, m = rel_l2(got, ref), max_rel(got, ref)
        assert e <= F32_ITER and m <= F32_ITER, (b, p.n, b % 3, batch.info[b], e, m)
    print(f"uneven batch: compared {len(pick)} problems, paths {sorted(paths)}")
