"""GPU tests of the batched plan: many uneven problems per launch.

A batch runs the same kernels as single-problem plans, so with the same
convolution path per problem the results are bitwise identical to the single
plans; every problem also matches the float64 oracle (1e-5 per apply, 1e-4
after iterations).  Problems with one kernel share its tables.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2505_22797_amd import mpik
from paper_2505_22797_amd import synth as S
from gpu_helpers import dev, rel_l2, rounded

pytestmark = pytest.mark.gpu


def _small_batch():
    specs = []
    shapes = [(24, 5, 3000, "direct", 0), (33, 12, 5000, "fft", 1), (48, 31, 9000, "fft", 2),
              (40, 9, 4000, "direct", 1), (64, 31, 12000, "direct", 0), (17, 16, 1500, "fft", 2)]
    for i, (n, R, t, mode, kind) in enumerate(shapes):
        if kind == 0:
            tr = S.lissajous(t, ax=0.85, ay=0.85)
        elif kind == 1:
            tr = S.lissajous(t, ax=0.8, ay=0.85, exc_amp=0.04, exc_cycles=17 * 30)
        else:
            tr = S.lissajous(t, ax=0.85, ay=0.85, t0=0.2, t1=0.75)
        specs.append(dict(n=n, h=S.h_fwhm2(n) * (0.9 + 0.05 * i), R=R, r=rounded(tr.r, torch.float32),
                          v=rounded(tr.v, torch.float32), c=rounded(S.ellipses_and_line(n, 1000 + i), torch.float32),
                          mode=mode))
    return specs


def _build(specs, tune=False, modes=True, columns=None):
    return mpik.Batch([(sp["n"], sp["h"], sp["R"], dev(sp["r"], torch.float32), dev(sp["v"], torch.float32),
                        sp["mode"] if modes else "auto") for sp in specs], tune=tune, columns=columns)


def _c_all(batch, specs):
    return torch.cat([dev(sp["c"], torch.float32).reshape(-1) for sp in specs])


def test_batch_equals_single_plans():
    """With the column kernels in the shape a single plan uses, every problem
    of the batch is bitwise the single-plan result."""
    specs = _small_batch()
    batch = _build(specs, columns="split")
    c_all = _c_all(batch, specs)
    s_all = batch.forward(c_all)
    rng = np.random.default_rng(0)
    y_all = dev(rounded(rng.standard_normal(batch.s_offsets[-1]), torch.float32), torch.float32)
    g_all = batch.adjoint(y_all)
    torch.cuda.synchronize()
    for b, sp in enumerate(specs):
        plan = mpik.Plan(sp["n"], sp["h"], sp["R"], dev(sp["r"], torch.float32), dev(sp["v"], torch.float32),
                         conv_mode=sp["mode"])
        assert batch.info[b]["conv_mode"] == sp["mode"] == plan.conv_mode
        s1 = plan.forward(dev(sp["c"], torch.float32))
        g1 = plan.adjoint(batch.s_views(y_all)[b].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(batch.s_views(s_all)[b], s1), b
        assert torch.equal(batch.c_views(g_all)[b], g1), b


def test_problems_with_one_kernel_share_its_tables():
    """Problems of a batch with the same N, R, h (and gradient and requested
    path) read one copy of the kernel tables: the plan is smaller than with
    distinct kernels by the duplicated spectra, twiddles and taps, and every
    problem -- those reading an earlier problem's tables included -- is
    bitwise its single-plan result and matches the oracle."""
    n, R, h = 64, 63, S.h_fwhm2(64)
    kinds = [dict(ax=0.85, ay=0.85), dict(ax=0.8, ay=0.85, exc_amp=0.04, exc_cycles=17 * 30),
             dict(ax=0.85, ay=0.85, t0=0.2, t1=0.75)]
    specs = []
    for i, (nn, RR, hh, t, mode, kind) in enumerate([(n, R, h, 5000, "fft", 0), (n, R, h, 7000, "fft", 1),
                                                      (n, R, 1.2 * h, 6000, "fft", 2), (n, R, h, 3000, "fft", 2),
                                                      (40, 9, S.h_fwhm2(40), 4000, "direct", 0),
                                                      (40, 9, S.h_fwhm2(40), 3500, "direct", 1)]):
        tr = S.lissajous(t, **kinds[kind])
        specs.append(dict(n=nn, h=hh, R=RR, r=rounded(tr.r, torch.float32), v=rounded(tr.v, torch.float32),
                          c=rounded(S.ellipses_and_line(nn, 2000 + i), torch.float32), mode=mode))
    batch = _build(specs, columns="split")
    distinct = [dict(sp, h=sp["h"] * (1.0 + 1e-3 * b)) for b, sp in enumerate(specs)]
    batch_d = _build(distinct, columns="split")
    H, W = 65, 19                       # M = 128 for N = 64, R = 63; direct window 2R + 1
    saved = batch_d.plan_mem.numel() - batch.plan_mem.numel()
    assert saved >= 2 * (3 * H * H * 4 + 128 * 8) + 3 * W * 20 * 4, saved
    c_all = _c_all(batch, specs)
    s_all = batch.forward(c_all)
    rng = np.random.default_rng(1)
    y_all = dev(rounded(rng.standard_normal(batch.s_offsets[-1]), torch.float32), torch.float32)
    g_all = batch.adjoint(y_all)
    torch.cuda.synchronize()
    for b, sp in enumerate(specs):
        plan = mpik.Plan(sp["n"], sp["h"], sp["R"], dev(sp["r"], torch.float32), dev(sp["v"], torch.float32),
                         conv_mode=sp["mode"])
        s1 = plan.forward(dev(sp["c"], torch.float32))
        g1 = plan.adjoint(batch.s_views(y_all)[b].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(batch.s_views(s_all)[b], s1), b
        assert torch.equal(batch.c_views(g_all)[b], g1), b
        M = O.Model(sp["n"], sp["h"], sp["R"], sp["r"], sp["v"])
        assert rel_l2(batch.s_views(s_all)[b].double().cpu().numpy(), M.forward(sp["c"])) <= 1e-5, b
    print(f"one kernel per group: plan {saved} bytes smaller than with distinct kernels", flush=True)
    batch.close()
    batch_d.close()


@pytest.mark.parametrize("columns", ["split", "wave"])
def test_batch_matches_oracle(columns):
    specs = _small_batch()
    batch = _build(specs, columns=columns)
    c_all = _c_all(batch, specs)
    s_all = batch.forward(c_all)
    rng = np.random.default_rng(1)
    y = rounded(rng.standard_normal(batch.s_offsets[-1]), torch.float32)
    g_all = batch.adjoint(dev(y, torch.float32))
    torch.cuda.synchronize()
    for b, sp in enumerate(specs):
        M = O.Model(sp["n"], sp["h"], sp["R"], sp["r"], sp["v"])
        s_ref = M.forward(sp["c"])
        assert rel_l2(batch.s_views(s_all)[b].double().cpu().numpy(), s_ref) <= 1e-5
        yb = y[batch.s_offsets[b]:batch.s_offsets[b + 1]].reshape(-1, 2)
        g_ref = M.adjoint(yb)
        assert rel_l2(batch.c_views(g_all)[b].double().cpu().numpy(), g_ref) <= 1e-5


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_wave_columns_full_kernel(dtype):
    """The column stages in the one-wave-per-column shape at M = 512, where
    every column transform is register-resident: three problems with full-size
    kernels (N + R > 256), among them a ragged last group of four columns
    (H = 257) and a grid far smaller than M, forward and transpose against
    the oracle in both precisions."""
    shapes = [(256, 255, 20000), (200, 199, 12000), (130, 129, 6000)]
    specs, models, cs, ys = [], [], [], []
    rng = np.random.default_rng(11)
    for i, (n, R, t) in enumerate(shapes):
        tr = S.lissajous(t, ax=0.85, ay=0.8 + 0.03 * i)
        r, v = rounded(tr.r, dtype), rounded(tr.v, dtype)
        h = S.h_fwhm2(n) * (0.95 + 0.05 * i)
        specs.append((n, h, R, dev(r, dtype), dev(v, dtype), "fft"))
        models.append(O.Model(n, h, R, r, v))
        cs.append(rounded(S.ellipses_and_line(n, 40 + i), dtype))
        ys.append(rounded(rng.standard_normal((t, 2)), dtype))
    batch = mpik.Batch(specs, dtype=dtype, tune=False, columns="wave")
    assert all(info["fft_size"] == 512 for info in batch.info)
    s_all = batch.forward(torch.cat([dev(c, dtype).reshape(-1) for c in cs]))
    g_all = batch.adjoint(torch.cat([dev(y, dtype).reshape(-1) for y in ys]))
    torch.cuda.synchronize()
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    for b, M in enumerate(models):
        assert rel_l2(batch.s_views(s_all)[b].double().cpu().numpy(), M.forward(cs[b])) <= tol, b
        assert rel_l2(batch.c_views(g_all)[b].double().cpu().numpy(), M.adjoint(ys[b])) <= tol, b


@pytest.mark.parametrize("denoise", [False, True])
def test_batch_iterate_matches_oracle(denoise):
    specs = _small_batch()[:4]
    batch = _build(specs)
    taus, s_list, models = [], [], []
    for sp in specs:
        M = O.Model(sp["n"], sp["h"], sp["R"], sp["r"], sp["v"])
        models.append(M)
        s_list.append(rounded(S.add_noise(M.forward(sp["c"]), 20.0, seed=1), torch.float32))
        taus.append(0.9 / O.power_lambda_max(M, iters=30))
    s_all = torch.cat([dev(s, torch.float32).reshape(-1) for s in s_list])
    c_all = torch.zeros(batch.c_offsets[-1], dtype=torch.float32, device="cuda")
    n_iter = 12
    sigma = 0.5 if denoise else 0.0
    batch.iterate(s_all, c_all, n_iter, taus, denoise_sigma_px=sigma, denoise_radius=2)
    torch.cuda.synchronize()
    for b, sp in enumerate(specs):
        ref = O.iterate(models[b], s_list[b], np.zeros((sp["n"], sp["n"])), taus[b], n_iter,
                        sigma_px=0.5 if denoise else None, radius=2)
        assert rel_l2(batch.c_views(c_all)[b].double().cpu().numpy(), ref) <= 1e-4, b


def test_uneven_batch_of_64_with_tuning():
    """64 problems: N from {64,...,256}, 10k-120k samples, Lissajous /
    perturbed / partial, h within +-20%, window R = 31; the autotuner picks the
    path per shape.  Every problem's forward and transpose match the oracle."""
    probs = S.batch_problems(64)
    specs = [dict(n=P.n, h=P.h, R=P.radius, r=rounded(P.traj.r, torch.float32), v=rounded(P.traj.v, torch.float32),
                  c=rounded(P.c, torch.float32), mode="auto") for P in probs]
    batch = _build(specs, tune=True, modes=False)
    c_all = _c_all(batch, specs)
    s_all = batch.forward(c_all)
    g_all = batch.adjoint(s_all)
    torch.cuda.synchronize()
    sv, gv = batch.s_views(s_all), batch.c_views(g_all)
    for b, sp in enumerate(specs):
        M = O.Model(sp["n"], sp["h"], sp["R"], sp["r"], sp["v"])
        s_ref = M.forward(sp["c"])
        s_got = sv[b].double().cpu().numpy()
        assert rel_l2(s_got, s_ref) <= 1e-5, (b, batch.info[b])
        g_ref = M.adjoint(rounded(s_got, torch.float32))
        assert rel_l2(gv[b].double().cpu().numpy(), g_ref) <= 1e-5, (b, batch.info[b])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_every_direct_slice_count_matches_oracle(dtype):
    """The autotuner's direct-path candidates, 4, 8 and 16 waves splitting a
    tile's window rows, each forced on a batch of direct-path problems: the
    forward, the transpose and three denoised iterations match the oracle,
    and the counts agree with each other to rounding."""
    shapes = [(24, 3, 2000), (40, 7, 4000), (33, 15, 3000), (64, 30, 6000)]
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    items = []
    for i, (n, R, t) in enumerate(shapes):
        tr = S.lissajous(t, ax=0.85, ay=0.8 + 0.01 * i)
        items.append(dict(n=n, R=R, h=S.h_fwhm2(n), r=rounded(tr.r, dtype), v=rounded(tr.v, dtype),
                          c=rounded(S.ellipses_and_line(n, 300 + i), dtype)))
    models = [O.Model(it["n"], it["h"], it["R"], it["r"], it["v"]) for it in items]
    taus = [0.9 / O.power_lambda_max(M, iters=20) for M in models]
    outs = {}
    for sl in (4, 8, 16):
        batch = mpik.Batch([(it["n"], it["h"], it["R"], dev(it["r"], dtype), dev(it["v"], dtype), "direct")
                            for it in items], dtype=dtype, tune=False, slices=sl)
        assert all(i["conv_mode"] == "direct" and i["slices"] == sl for i in batch.info)
        c_all = torch.cat([dev(it["c"], dtype).reshape(-1) for it in items])
        s_all = batch.forward(c_all)
        g_all = batch.adjoint(s_all)
        x_all = torch.zeros_like(c_all)
        batch.iterate(s_all, x_all, 3, taus, 0.5, 2)
        torch.cuda.synchronize()
        outs[sl] = [[x.double().cpu().numpy() for x in batch.s_views(s_all)],
                    [x.double().cpu().numpy() for x in batch.c_views(g_all)],
                    [x.double().cpu().numpy() for x in batch.c_views(x_all)]]
        batch.close()
        for b, (it, M) in enumerate(zip(items, models)):
            s_ref = M.forward(it["c"])
            s_got = outs[sl][0][b]
            assert rel_l2(s_got, s_ref) <= tol, (sl, b)
            assert rel_l2(outs[sl][1][b], M.adjoint(rounded(s_got, dtype))) <= tol, (sl, b)
            x_ref = O.iterate(M, rounded(s_got, dtype), np.zeros((it["n"], it["n"])), taus[b], 3, sigma_px=0.5,
                              radius=2)
            assert rel_l2(outs[sl][2][b], x_ref) <= 10 * tol, (sl, b)
    for k in range(3):
        for b in range(len(items)):
            assert rel_l2(outs[4][k][b], outs[16][k][b]) <= tol, (k, b)


@pytest.mark.parametrize("columns", ["split", "wave"])
def test_uneven_sizes_iterate_matches_oracle(columns):
    """Problems of very different sizes in one batch: every launch is sized
    for the largest one, so the block-to-row mapping of the small ones must
    stay one-to-one (the in-place gradient step would otherwise be applied
    twice)."""
    specs = []
    for i, (n, R, t) in enumerate([(200, 31, 20000), (24, 23, 3000), (72, 40, 8000), (9, 8, 500)]):
        tr = S.lissajous(t, ax=0.8, ay=0.8)
        specs.append(dict(n=n, h=S.h_fwhm2(n), R=R, r=rounded(tr.r, torch.float32), v=rounded(tr.v, torch.float32),
                          c=rounded(S.blobs(n, 40 + i), torch.float32), mode="fft"))
    batch = _build(specs, columns=columns)
    taus, s_list, models = [], [], []
    for sp in specs:
        M = O.Model(sp["n"], sp["h"], sp["R"], sp["r"], sp["v"])
        models.append(M)
        s_list.append(rounded(M.forward(sp["c"]), torch.float32))
        taus.append(0.9 / O.power_lambda_max(M, iters=20))
    s_all = torch.cat([dev(s, torch.float32).reshape(-1) for s in s_list])
    c_all = torch.zeros(batch.c_offsets[-1], dtype=torch.float32, device="cuda")
    batch.iterate(s_all, c_all, 6, taus)
    torch.cuda.synchronize()
    for b, sp in enumerate(specs):
        ref = O.iterate(models[b], s_list[b], np.zeros((sp["n"], sp["n"])), taus[b], 6)
        assert rel_l2(batch.c_views(c_all)[b].double().cpu().numpy(), ref) <= 1e-4, b


def _chunk_specs(shapes, seed):
    specs = []
    for i, (n, R, t, mode) in enumerate(shapes):
        tr = S.lissajous(t, ax=0.85 - 0.01 * (i % 5), ay=0.85)
        specs.append(dict(n=n, h=S.h_fwhm2(n) * (0.9 + 0.01 * i), R=R, r=rounded(tr.r, torch.float32),
                          v=rounded(tr.v, torch.float32), c=rounded(S.blobs(n, seed + i), torch.float32), mode=mode))
    return specs


CHUNKED = {
    # 17 problems of one FFT size: each launch sequence splits into four problem ranges on side streams
    "one_size": [(24 + (i % 3), 5 + i % 4, 1500 + 100 * i, "fft") for i in range(17)],
    # 18 problems, two FFT sizes and two direct problems: two ranges per size, the direct path beside them
    "two_sizes": [(24, 7, 2000, "fft"), (48, 31, 5000, "fft")] * 8 + [(20, 4, 1200, "direct"), (28, 6, 1800, "direct")],
    # 49 problems of one FFT size: two problem ranges of uneven length (24 and 25)
    "many_one_size": [(20 + (i % 5), 4 + i % 3, 600 + 20 * i, "fft") for i in range(49)],
}


@pytest.mark.parametrize("kind", sorted(CHUNKED))
def test_chunked_batch_equals_single_plans(kind):
    """Batches of at least 16 problems run each FFT size group as several
    problem ranges on side streams; every problem is still bitwise the
    single-plan result (column kernels in the single-plan shape), and the
    pair call bitwise the forward and transpose calls."""
    specs = _chunk_specs(CHUNKED[kind], 300)
    batch = _build(specs, columns="split")
    c_all = _c_all(batch, specs)
    s_all = batch.forward(c_all)
    rng = np.random.default_rng(5)
    y_all = dev(rounded(rng.standard_normal(batch.s_offsets[-1]), torch.float32), torch.float32)
    g_all = batch.adjoint(y_all)
    # the pair call gives the two separate calls' results, bitwise
    s_p, g_p = batch.pair(c_all)
    g_sep = batch.adjoint(s_all)
    torch.cuda.synchronize()
    assert torch.equal(s_p, s_all) and torch.equal(g_p, g_sep)
    for b, sp in enumerate(specs):
        plan = mpik.Plan(sp["n"], sp["h"], sp["R"], dev(sp["r"], torch.float32), dev(sp["v"], torch.float32),
                         conv_mode=sp["mode"])
        s1 = plan.forward(dev(sp["c"], torch.float32))
        g1 = plan.adjoint(batch.s_views(y_all)[b].contiguous())
        s2, g2 = plan.pair(dev(sp["c"], torch.float32))
        torch.cuda.synchronize()
        assert torch.equal(batch.s_views(s_all)[b], s1), b
        assert torch.equal(batch.c_views(g_all)[b], g1), b
        assert torch.equal(s2, s1) and torch.equal(g2, plan.adjoint(s1)), b


@pytest.mark.parametrize("kind", sorted(CHUNKED))
def test_chunked_batch_iterate_matches_oracle(kind):
    """The per-problem step tau_b follows its problem into its range: a
    different tau per problem, 10 iterations (one captured block of eight,
    then two single ones), each against the oracle."""
    specs = _chunk_specs(CHUNKED[kind], 400)
    batch = _build(specs)
    taus, s_list, models = [], [], []
    for i, sp in enumerate(specs):
        M = O.Model(sp["n"], sp["h"], sp["R"], sp["r"], sp["v"])
        models.append(M)
        s_list.append(rounded(M.forward(sp["c"]), torch.float32))
        taus.append((0.5 + 0.02 * i) / O.power_lambda_max(M, iters=20))
    s_all = torch.cat([dev(s, torch.float32).reshape(-1) for s in s_list])
    c_all = torch.zeros(batch.c_offsets[-1], dtype=torch.float32, device="cuda")
    batch.iterate(s_all, c_all, 10, taus)
    torch.cuda.synchronize()
    for b, sp in enumerate(specs):
        ref = O.iterate(models[b], s_list[b], np.zeros((sp["n"], sp["n"])), taus[b], 10)
        assert rel_l2(batch.c_views(c_all)[b].double().cpu().numpy(), ref) <= 1e-4, b


def test_pair_in_a_captured_graph_replays_like_eager():
    """The pair call of a batch split into problem ranges (side streams
    forked and joined inside the call), captured in a graph: three replays,
    each after new inputs are copied in and other eager work has run, equal
    the eager results bitwise."""
    specs = _chunk_specs(CHUNKED["one_size"], 700)
    batch = _build(specs, columns="wave")
    n_c, n_s = batch.c_offsets[-1], batch.s_offsets[-1]
    c_in = torch.empty(n_c, dtype=torch.float32, device="cuda")
    s_out = torch.empty(n_s, dtype=torch.float32, device="cuda")
    g_out = torch.empty(n_c, dtype=torch.float32, device="cuda")
    c_in.copy_(_c_all(batch, specs))
    batch.pair(c_in, s_out, g_out)                 # warm: workspaces
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.pair(c_in, s_out, g_out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.pair(c_in, s_out, g_out)
    rng = np.random.default_rng(9)
    for rep in range(3):
        x = torch.tensor(rounded(rng.standard_normal(n_c), torch.float32), dtype=torch.float32, device="cuda")
        s_ref, g_ref = batch.pair(x)              # eager, other buffers
        torch.cuda.synchronize()
        c_in.copy_(x)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(s_out, s_ref) and torch.equal(g_out, g_ref), rep
