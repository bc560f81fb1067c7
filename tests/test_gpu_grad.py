"""GPU parity of the differentiation layer: the derivative kernels through the
C ABI, the autograd Functions and the checkpointed unrolled solve against the
float64 oracle (whose own derivatives are pinned to finite differences in
test_oracle_grad.py).

The trajectory of problem b is (ax_b rho_x, ay_b rho_y) with velocities
(ax_b nu_x, ay_b nu_y).  The library scales the unit shapes in the compute
precision; the oracle is given the same rounded positions (float32 products of
float32 values are correctly rounded on both sides), so both use the same base
cells, and the unrolled-gradient oracle keeps those cells frozen.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2505_22797_amd import autograd as AG
from paper_2505_22797_amd import mpik
from paper_2505_22797_amd import synth as S
from gpu_helpers import dev, rel_l2, rounded

pytestmark = pytest.mark.gpu

NP = {torch.float32: np.float32, torch.float64: np.float64}
APPLY_TOL = {torch.float32: 1e-5, torch.float64: 1e-12}


class GradCase:
    """Problems with unit trajectory shapes, amplitudes and phantoms, prepared
    for both sides."""

    def __init__(self, shapes, dtype, seed=0, amp=(0.85, 0.8), interp="bilinear"):
        self.dtype = dtype
        self.interp = interp
        self.items = []
        for i, (n, R, t, mode) in enumerate(shapes):
            tr = S.lissajous(t, ax=1.0, ay=1.0)
            rho = rounded(tr.r, dtype)
            nu = rounded(tr.v, dtype)
            ax, ay = (float(NP[dtype](a * (1.0 + 0.01 * i))) for a in amp)
            r = (rho.astype(NP[dtype]) * NP[dtype](np.array([ax, ay]))).astype(np.float64)
            v = (nu.astype(NP[dtype]) * NP[dtype](np.array([ax, ay]))).astype(np.float64)
            h = S.h_fwhm2(n) * (1.0 + 0.1 * i)
            self.items.append(dict(n=n, R=R, t=t, mode=mode, rho=rho, nu=nu, ax=ax, ay=ay, r=r, v=v, h=h,
                                   model=O.Model(n, h, R, r, v, interp=interp),
                                   c=rounded(S.blobs(n, seed + i), dtype)))
        self.op = AG.TrajectoryOperator([it["n"] for it in self.items], [it["R"] for it in self.items],
                                        [dev(it["rho"], dtype) for it in self.items],
                                        [dev(it["nu"], dtype) for it in self.items], dtype=dtype,
                                        conv_mode=self.items[0]["mode"], interp=interp)
        self.h = torch.tensor([it["h"] for it in self.items], dtype=torch.float64)
        self.ax = torch.tensor([it["ax"] for it in self.items], dtype=torch.float64)
        self.ay = torch.tensor([it["ay"] for it in self.items], dtype=torch.float64)

    def plan(self):
        return self.op.plan(self.h, self.ax, self.ay)

    def cat(self, arrays):
        return torch.cat([dev(rounded(a, self.dtype), self.dtype).reshape(-1) for a in arrays])

    @staticmethod
    def split(plan, flat, space):
        torch.cuda.synchronize()
        views = plan.c_views(flat) if space == "grid" else plan.s_views(flat)
        return [x.double().cpu().numpy() for x in views]


SHAPES = [(32, 7, 2500, "direct"), (48, 15, 5000, "direct"), (40, 12, 3001, "direct")]
SHAPES_WIDE = [(32, 7, 2500, "direct"), (48, 31, 5000, "direct"), (64, 31, 8000, "direct")]
SHAPES_FFT = [(32, 7, 2500, "fft"), (48, 31, 5000, "fft"), (40, 12, 3001, "fft")]


# the float64 direct path keeps its input tile in LDS, which limits it to R <= 30
@pytest.mark.parametrize("dtype,shapes,interp", [
    (torch.float32, SHAPES, "bilinear"), (torch.float64, SHAPES, "bilinear"), (torch.float32, SHAPES_WIDE, "bilinear"),
    (torch.float32, SHAPES_FFT, "bilinear"), (torch.float64, SHAPES_FFT, "bilinear"),
    (torch.float32, SHAPES_FFT, "cosine"), (torch.float64, SHAPES, "cosine"), (torch.float64, SHAPES_FFT, "cosine")],
    ids=["direct-f32", "direct-f64", "direct63-f32", "fft-f32", "fft-f64", "fft-f32-cos", "direct-f64-cos",
         "fft-f64-cos"])
def test_derivative_blocks_match_oracle(dtype, shapes, interp):
    gc = GradCase(shapes, dtype, interp=interp)
    plan = gc.plan()
    tol = APPLY_TOL[dtype]
    rng = np.random.default_rng(5)
    ys = [rounded(rng.standard_normal((it["t"], 2)), dtype) for it in gc.items]
    xs = [it["c"] for it in gc.items]
    x_all, y_all = gc.cat(xs), gc.cat(ys)

    dh = GradCase.split(plan, plan.forward_dh(x_all), "signal")
    res = GradCase.split(plan, plan.residual(x_all, y_all), "signal")
    g_r, g_v = plan.traj_vjp(x_all, y_all)
    g_r, g_v = GradCase.split(plan, g_r, "signal"), GradCase.split(plan, g_v, "signal")
    taus = [0.3, 0.7, 1.1]
    step = GradCase.split(plan, plan.adjoint_step(y_all, x_all, taus), "grid")
    den = GradCase.split(plan, plan.denoise(x_all, 0.5, 2), "grid")
    for b, it in enumerate(gc.items):
        M = it["model"]
        assert rel_l2(dh[b], M.forward_dh(xs[b])) <= tol, ("forward_dh", b)
        assert rel_l2(res[b], M.forward(xs[b]) - ys[b]) <= tol, ("residual", b)
        r_ref, v_ref = M.traj_vjp(xs[b], ys[b])
        assert rel_l2(g_r[b], r_ref) <= tol, ("g_r", b)
        assert rel_l2(g_v[b], v_ref) <= tol, ("g_v", b)
        assert rel_l2(step[b], xs[b] - taus[b] * M.adjoint(ys[b])) <= tol, ("adjoint_step", b)
        assert rel_l2(den[b], O.denoise(xs[b], 0.5, 2)) <= tol, ("denoise", b)


@pytest.mark.parametrize("dtype,shapes", [(torch.float32, SHAPES_FFT), (torch.float64, SHAPES)], ids=["fft-f32", "direct-f64"])
def test_composite_vjps_are_their_building_blocks(dtype, shapes):
    """mpi_vjp_forward and mpi_vjp_adjoint against the building-block calls
    they compose, bit for bit, and against the oracle's VJPs of s = A c and
    c' = A^T y (the h component through its definition <(dA/dh) x, y>)."""
    gc = GradCase(shapes, dtype)
    plan = gc.plan()
    rng = np.random.default_rng(17)
    ys = [rounded(rng.standard_normal((it["t"], 2)), dtype) for it in gc.items]
    xs = [it["c"] for it in gc.items]
    x_all, y_all = gc.cat(xs), gc.cat(ys)
    # s = A c with upstream gradient y; c' = A^T y with upstream gradient x
    gcx, gh_f, gr_f, gv_f = plan.vjp_forward(x_all, y_all)
    gy, gh_a, gr_a, gv_a = plan.vjp_adjoint(y_all, x_all)
    ref_gc = plan.adjoint(y_all)
    ref_gy = plan.forward(x_all)
    ref_gh = plan.dot(plan.forward_dh(x_all), y_all)
    ref_gr, ref_gv = plan.traj_vjp(x_all, y_all)
    torch.cuda.synchronize()
    for got, ref in ((gcx, ref_gc), (gy, ref_gy), (gh_f, ref_gh), (gh_a, ref_gh), (gr_f, ref_gr), (gv_f, ref_gv),
                     (gr_a, ref_gr), (gv_a, ref_gv)):
        assert torch.equal(got, ref)
    tol = APPLY_TOL[dtype]
    g_r, g_v = GradCase.split(plan, gr_f, "signal"), GradCase.split(plan, gv_f, "signal")
    gh = gh_f.cpu().numpy()
    for b, it in enumerate(gc.items):
        M = it["model"]
        r_ref, v_ref = M.traj_vjp(xs[b], ys[b])
        assert rel_l2(g_r[b], r_ref) <= tol and rel_l2(g_v[b], v_ref) <= tol, b
        h_ref = np.sum(M.forward_dh(xs[b]) * ys[b])
        assert abs(gh[b] - h_ref) <= tol * np.sum(np.abs(M.forward_dh(xs[b]) * ys[b])), b
    with pytest.raises(ValueError):
        plan.vjp_forward(x_all, x_all)               # an upstream gradient of the wrong shape


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_dot_is_exact_per_problem(dtype):
    """Per-problem float64 sums of products, per component and over the grid."""
    gc = GradCase(SHAPES, dtype)
    plan = gc.plan()
    rng = np.random.default_rng(9)
    a = [rounded(rng.standard_normal((it["t"], 2)), dtype) for it in gc.items]
    b = [rounded(rng.standard_normal((it["t"], 2)), dtype) for it in gc.items]
    p = [rounded(rng.standard_normal((it["n"], it["n"])), dtype) for it in gc.items]
    q = [rounded(rng.standard_normal((it["n"], it["n"])), dtype) for it in gc.items]
    got = {k: plan.dot(gc.cat(a), gc.cat(b), comp=k).cpu().numpy() for k in ("x", "y", "both")}
    grid = plan.dot(gc.cat(p), gc.cat(q), space="grid").cpu().numpy()
    for i in range(len(gc.items)):
        ref = {"x": np.sum(a[i][:, 0] * b[i][:, 0]), "y": np.sum(a[i][:, 1] * b[i][:, 1]),
               "both": np.sum(a[i] * b[i])}
        for k in ref:
            assert abs(got[k][i] - ref[k]) <= 1e-13 * np.sum(np.abs(a[i] * b[i])), (k, i)
        assert abs(grid[i] - np.sum(p[i] * q[i])) <= 1e-13 * np.sum(np.abs(p[i] * q[i])), i


def test_scale_trajectory_rounds_once():
    """r = (ax rho_x, ay rho_y), v = (ax nu_x, ay nu_y): each product formed in
    float64 and rounded once, bitwise, in both dtypes."""
    rng = np.random.default_rng(21)
    for dtype, npd in ((torch.float32, np.float32), (torch.float64, np.float64)):
        rho = rng.standard_normal((5001, 2)).astype(npd)
        nu = (50.0 * rng.standard_normal((5001, 2))).astype(npd)
        ax, ay = 0.8819, 1.0234567
        r, v = mpik.scale_trajectory(torch.tensor(rho, device="cuda"), torch.tensor(nu, device="cuda"), ax, ay)
        torch.cuda.synchronize()
        amp = np.array([ax, ay])
        assert np.array_equal(r.cpu().numpy(), (rho.astype(np.float64) * amp).astype(npd))
        assert np.array_equal(v.cpu().numpy(), (nu.astype(np.float64) * amp).astype(npd))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_reduce_lissajous_is_exact_per_problem(dtype):
    """The amplitude chain rule of the library, per problem: sum_k g_r,x rho_x +
    g_v,x nu_x (and y) in float64 against the float64 sums of the same values,
    bitwise repeatable."""
    gc = GradCase(SHAPES, dtype)
    plan = gc.plan()
    rng = np.random.default_rng(23)
    g_r, g_v, rho, nu = ([rounded(rng.standard_normal((it["t"], 2)), dtype) for it in gc.items] for _ in range(4))
    args = [gc.cat(x) for x in (g_r, g_v, rho, nu)]
    gax, gay = plan.reduce_lissajous(*args)
    gax2, gay2 = plan.reduce_lissajous(*args)
    gax, gay = gax.cpu().numpy(), gay.cpu().numpy()
    assert np.array_equal(gax, gax2.cpu().numpy()) and np.array_equal(gay, gay2.cpu().numpy())
    for i in range(len(gc.items)):
        for c, got in ((0, gax[i]), (1, gay[i])):
            terms = g_r[i][:, c] * rho[i][:, c] + g_v[i][:, c] * nu[i][:, c]
            assert abs(got - np.sum(terms)) <= 1e-13 * np.sum(np.abs(terms)), (i, c)


def _param_grads_ref(it, x, y):
    """Oracle gradients of <y, A x> with respect to h, ax, ay."""
    M = it["model"]
    gh = np.sum(M.forward_dh(x) * y)
    g_r, g_v = M.traj_vjp(x, y)
    gax = np.sum(g_r[:, 0] * it["rho"][:, 0]) + np.sum(g_v[:, 0] * it["nu"][:, 0])
    gay = np.sum(g_r[:, 1] * it["rho"][:, 1]) + np.sum(g_v[:, 1] * it["nu"][:, 1])
    return gh, gax, gay


def _close(got, ref, tol, scale=None):
    return abs(got - ref) <= tol * (abs(ref) if scale is None else scale)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_autograd_apply_and_transpose_match_oracle(dtype):
    gc = GradCase(SHAPES_FFT, dtype)
    tol = 10 * APPLY_TOL[dtype]
    rng = np.random.default_rng(11)
    ws = [rounded(rng.standard_normal((it["t"], 2)), dtype) for it in gc.items]
    xs = [it["c"] for it in gc.items]
    # s = A c, L = <w, s>
    c_all = gc.cat(xs).requires_grad_(True)
    h, ax, ay = (t.clone().requires_grad_(True) for t in (gc.h, gc.ax, gc.ay))
    s_all = AG.apply_A(gc.op, c_all, h, ax, ay)
    loss = torch.sum(s_all.double() * gc.cat(ws).double())
    g_c, g_h, g_ax, g_ay = torch.autograd.grad(loss, (c_all, h, ax, ay))
    plan = gc.plan()
    g_c = GradCase.split(plan, g_c.detach(), "grid")
    for b, it in enumerate(gc.items):
        assert rel_l2(g_c[b], it["model"].adjoint(ws[b])) <= APPLY_TOL[dtype], b
        ref = _param_grads_ref(it, xs[b], ws[b])
        for got, r_, name in zip((g_h[b], g_ax[b], g_ay[b]), ref, ("h", "ax", "ay")):
            assert _close(float(got), r_, tol), (name, b, float(got), r_)
    # c' = A^T y, L = <p, c'>
    ps = [rounded(rng.standard_normal((it["n"], it["n"])), dtype) for it in gc.items]
    y_all = gc.cat(ws).requires_grad_(True)
    h, ax, ay = (t.clone().requires_grad_(True) for t in (gc.h, gc.ax, gc.ay))
    c_out = AG.apply_AT(gc.op, y_all, h, ax, ay)
    loss = torch.sum(c_out.double() * gc.cat(ps).double())
    g_y, g_h, g_ax, g_ay = torch.autograd.grad(loss, (y_all, h, ax, ay))
    g_y = GradCase.split(plan, g_y.detach(), "signal")
    for b, it in enumerate(gc.items):
        assert rel_l2(g_y[b], it["model"].forward(ps[b])) <= APPLY_TOL[dtype], b
        ref = _param_grads_ref(it, ps[b], ws[b])
        for got, r_, name in zip((g_h[b], g_ax[b], g_ay[b]), ref, ("h", "ax", "ay")):
            assert _close(float(got), r_, tol), (name, b, float(got), r_)


def _unrolled_setup(gc, snr_db=20.0, h_scale=1.05, a_scale=0.98, power_iters=20):
    """Measurements from the nominal operator plus noise; the reconstruction
    runs at perturbed parameters with a fixed step 0.9 / lambda_max."""
    s_list, taus, truths = [], [], []
    for it in gc.items:
        nominal = O.Model(it["n"], it["h"] / h_scale, it["R"], it["r"] / a_scale, it["v"] / a_scale)
        truths.append(it["c"])
        s_list.append(rounded(S.add_noise(nominal.forward(it["c"]), snr_db, seed=7), gc.dtype))
        taus.append(0.9 / O.power_lambda_max(it["model"], iters=power_iters))
    return s_list, taus, truths


def _unrolled_gpu(gc, s_list, taus, truths, n_iter, sigma, every):
    c0 = torch.zeros(sum(it["n"] ** 2 for it in gc.items), dtype=gc.dtype, device="cuda", requires_grad=True)
    h, ax, ay = (t.clone().requires_grad_(True) for t in (gc.h, gc.ax, gc.ay))
    c_k = AG.unrolled_solve(gc.op, gc.cat(s_list), c0, h, ax, ay, taus, n_iter=n_iter, sigma_px=sigma,
                            radius=2, every=every)
    loss = torch.sum((c_k.double() - gc.cat(truths).double()) ** 2)
    g_c0, g_h, g_ax, g_ay = torch.autograd.grad(loss, (c0, h, ax, ay))
    views = GradCase.split(gc.plan(), g_c0.detach(), "grid")
    return float(loss.detach()), views, g_h.numpy(), g_ax.numpy(), g_ay.numpy()


def _unrolled_ref(it, s, tau, c_true, n_iter, sigma, **kw):
    a = dict(h=it["h"], ax=it["ax"], ay=it["ay"])
    a.update(kw)
    return O.unrolled_gradients(it["n"], a["h"], it["R"], a["ax"], a["ay"], it["rho"], it["nu"], s, c_true,
                                np.zeros((it["n"], it["n"])), tau, n_iter, sigma_px=sigma,
                                frozen=it["model"].cells(), interp=it["model"].interp)


SHAPES_MIXED = [(32, 7, 2500, "auto"), (48, 31, 5000, "auto"), (40, 12, 3001, "auto")]   # direct + FFT


@pytest.mark.parametrize("dtype,sigma,shapes,interp", [
    (torch.float32, None, SHAPES_FFT, "bilinear"), (torch.float32, 0.5, SHAPES_FFT, "bilinear"),
    (torch.float64, 0.5, SHAPES_FFT, "bilinear"), (torch.float32, 0.5, SHAPES, "bilinear"),
    (torch.float64, None, SHAPES, "bilinear"), (torch.float32, 0.5, SHAPES_MIXED, "bilinear"),
    (torch.float32, 0.5, SHAPES_MIXED, "cosine"), (torch.float64, 0.5, SHAPES_MIXED, "cosine")],
    ids=["fft-f32", "fft-f32-den", "fft-f64-den", "direct-f32-den", "direct-f64", "mixed-f32-den",
         "mixed-f32-den-cos", "mixed-f64-den-cos"])
def test_unrolled_gradients_match_oracle(dtype, sigma, shapes, interp):
    """K = 7 with checkpoints every 3 (a ragged last segment), three problems
    of different sizes in one batch."""
    gc = GradCase(shapes, dtype, interp=interp)
    if shapes is SHAPES_MIXED:
        assert {inf["conv_mode"] for inf in gc.plan().info} == {"direct", "fft"}
    s_list, taus, truths = _unrolled_setup(gc)
    K = 7
    loss, g_c0, g_h, g_ax, g_ay = _unrolled_gpu(gc, s_list, taus, truths, K, sigma, every=3)
    tol = 1e-4 if dtype == torch.float32 else 1e-9
    total = 0.0
    for b, it in enumerate(gc.items):
        l_ref, g = _unrolled_ref(it, s_list[b], taus[b], truths[b], K, sigma)
        total += l_ref
        assert rel_l2(g_c0[b], g["c0"]) <= tol, ("c0", b)
        for got, name in ((g_h[b], "h"), (g_ax[b], "ax"), (g_ay[b], "ay")):
            assert _close(got, g[name], tol), (name, b, got, g[name])
    assert _close(loss, total, tol)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_unrolled_gradients_do_not_depend_on_checkpoint_spacing(dtype):
    """One segment, segments of one step, and a ragged split agree: the reverse
    sweep recomputes each segment from its checkpoint."""
    gc = GradCase(SHAPES_MIXED, dtype)
    s_list, taus, truths = _unrolled_setup(gc)
    runs = [_unrolled_gpu(gc, s_list, taus, truths, 6, 0.5, every=e) for e in (6, 1, 4)]
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    for other in runs[1:]:
        for b in range(len(gc.items)):
            assert rel_l2(other[1][b], runs[0][1][b]) <= tol
        for i in (2, 3, 4):
            assert np.all(np.abs(other[i] - runs[0][i]) <= tol * np.abs(runs[0][i]))


def _oracle_loss(it, s, tau, c_true, n_iter, sigma, **kw):
    """The oracle's loss |c_K - c_true|^2 with the base cells frozen."""
    a = dict(h=it["h"], ax=it["ax"], ay=it["ay"])
    a.update(kw)
    scale = np.array([a["ax"], a["ay"]])
    M = O.Model(it["n"], a["h"], it["R"], it["rho"] * scale, it["nu"] * scale, frozen=it["model"].cells())
    c = O.iterate(M, s, np.zeros((it["n"], it["n"])), tau, n_iter, sigma_px=sigma, radius=2)
    return float(np.sum((c - c_true) ** 2))


def test_differentiation_workload_matches_oracle_and_finite_differences():
    """8 problems at 256^2, 53,856 samples, 63x63 window, K = 20 with
    checkpoints every 5, denoising on; measurements at the nominal parameters
    plus 20 dB noise, reconstruction at h x 1.05 and amplitudes x 0.98.  Two
    problems are compared with the oracle's gradients, and for one of them the
    scalar gradients also with float64 central differences of the oracle's
    loss (base cells frozen)."""
    probs = S.gradient_problems(8)
    n, R, T = probs[0].n, probs[0].radius, probs[0].n_samples
    assert (n, R, T) == (256, 31, 53856)
    dtype = torch.float32
    amp = float(np.float32(S.AMPLITUDE * 0.98))
    gc = GradCase([(n, R, T, "fft")] * 8, dtype, amp=(amp, amp))
    checked = (0, 5)
    for b, (it, P) in enumerate(zip(gc.items, probs)):
        # one operator for all eight problems (h, trajectory); the phantoms differ
        it["h"] = P.h * 1.05
        it["ax"] = it["ay"] = amp
        it["r"] = (it["rho"].astype(np.float32) * np.float32(amp)).astype(np.float64)
        it["v"] = (it["nu"].astype(np.float32) * np.float32(amp)).astype(np.float64)
        it["c"] = rounded(P.c, dtype)
        it["model"] = O.Model(n, it["h"], R, it["r"], it["v"]) if b in checked else None
    gc.h = torch.tensor([it["h"] for it in gc.items], dtype=torch.float64)
    gc.ax = torch.tensor([amp] * 8, dtype=torch.float64)
    gc.ay = gc.ax.clone()
    nominal = O.Model(n, probs[0].h, R, gc.items[0]["rho"] * S.AMPLITUDE, gc.items[0]["nu"] * S.AMPLITUDE)
    s_list = [rounded(S.add_noise(nominal.forward(it["c"]), 20.0, seed=P.seed), dtype)
              for it, P in zip(gc.items, probs)]
    tau = 0.9 / O.power_lambda_max(gc.items[0]["model"], iters=15)
    truths = [it["c"] for it in gc.items]
    K, sigma = 20, 0.5
    _, g_c0, g_h, g_ax, g_ay = _unrolled_gpu(gc, s_list, [tau] * 8, truths, K, sigma, every=5)
    for b in checked:
        _, g = _unrolled_ref(gc.items[b], s_list[b], tau, truths[b], K, sigma)
        assert rel_l2(g_c0[b], g["c0"]) <= 1e-4, ("c0", b)
        for got, name in ((g_h[b], "h"), (g_ax[b], "ax"), (g_ay[b], "ay")):
            assert _close(got, g[name], 1e-4), (name, b, got, g[name])
    # float64 central differences of the oracle's loss, cells frozen (the
    # derivative inside every sample's bilinear patch)
    it = gc.items[0]
    crossed = 0
    for name, got in (("h", g_h[0]), ("ax", g_ax[0]), ("ay", g_ay[0])):
        val = it[name]
        e = 1e-6 * val
        fd = (_oracle_loss(it, s_list[0], tau, truths[0], K, sigma, **{name: val + e})
              - _oracle_loss(it, s_list[0], tau, truths[0], K, sigma, **{name: val - e})) / (2 * e)
        assert _close(got, fd, 1e-4), (name, got, fd)
        if name != "h":
            k = 0 if name == "ax" else 1
            g0 = (it["rho"][:, k] * val + 1.0) * (n / 2.0) - 0.5
            g1 = (it["rho"][:, k] * (val + e) + 1.0) * (n / 2.0) - 0.5
            crossed += int(np.sum(np.floor(g0) != np.floor(g1)))
    print(f"samples whose base cell a +1e-6 relative amplitude step moves: {crossed}")


def test_cosine_unrolled_gradients_match_unfrozen_finite_differences():
    """Under the cosine interpolator the signal is C^1 in the sample
    positions, so central differences of the oracle's loss taken without
    freezing the base cells (samples may change cells within the step) agree
    with the library's gradients; 64^2, 15x15 window, K = 6, every 4."""
    dtype = torch.float64
    gc = GradCase([(64, 15, 9000, "fft")], dtype, interp="cosine")
    s_list, taus, truths = _unrolled_setup(gc)
    K, sigma = 6, 0.5
    _, _, g_h, g_ax, g_ay = _unrolled_gpu(gc, s_list, taus, truths, K, sigma, every=4)
    it = gc.items[0]

    def loss(**kw):
        a = dict(h=it["h"], ax=it["ax"], ay=it["ay"])
        a.update(kw)
        scale = np.array([a["ax"], a["ay"]])
        M = O.Model(it["n"], a["h"], it["R"], it["rho"] * scale, it["nu"] * scale, interp="cosine")
        c = O.iterate(M, s_list[0], np.zeros((it["n"], it["n"])), taus[0], K, sigma_px=sigma, radius=2)
        return float(np.sum((c - truths[0]) ** 2))

    crossed = 0
    for name, got in (("h", g_h[0]), ("ax", g_ax[0]), ("ay", g_ay[0])):
        val = it[name]
        # a step across a node meets a jump of the second derivative, which
        # makes the difference first order in the step there: 1e-5 relative
        # keeps that error near 1e-6 while samples still change cells
        e = 1e-5 * val
        fd = (loss(**{name: val + e}) - loss(**{name: val - e})) / (2 * e)
        assert _close(got, fd, 1e-5), (name, got, fd)
        if name != "h":
            k = 0 if name == "ax" else 1
            g0 = (it["rho"][:, k] * (val - e) + 1.0) * (it["n"] / 2.0) - 0.5
            g1 = (it["rho"][:, k] * (val + e) + 1.0) * (it["n"] / 2.0) - 0.5
            crossed += int(np.sum(np.floor(g0) != np.floor(g1)))
    assert crossed > 0, crossed        # some samples change cells within the steps
