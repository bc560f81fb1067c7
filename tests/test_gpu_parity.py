"""GPU parity: the HIP path through the C ABI against the float64 oracle.

Tolerances (relative L2 over the whole output): 1e-12 per apply in float64,
1e-5 per apply in float32, 1e-10 after 50 float64 Landweber iterations and
1e-4 after the float32 iterations.  Inputs are generated in float64 and
rounded once to the compute precision; the oracle consumes the rounded
values.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2505_22797_amd import mpik
from paper_2505_22797_amd import synth as S
from gpu_helpers import Case, case_from, rel_l2

pytestmark = pytest.mark.gpu

F64_APPLY = 1e-12
F32_APPLY = 1e-5


def _check_apply(cs: Case, tol, seed=0):
    rng = np.random.default_rng(seed)
    s_ref = cs.model.forward(cs.c)
    s = cs.plan.forward(cs.t(cs.c))
    e_fwd = rel_l2(Case.host(s), s_ref)
    y = rng.standard_normal(s_ref.shape)
    y = np.asarray(y, dtype=np.float32 if cs.dtype == torch.float32 else np.float64).astype(np.float64)
    c_ref = cs.model.adjoint(y)
    c = cs.plan.adjoint(cs.t(y))
    e_adj = rel_l2(Case.host(c), c_ref)
    assert e_fwd <= tol, f"forward rel-L2 {e_fwd:.3e}"
    assert e_adj <= tol, f"adjoint rel-L2 {e_adj:.3e}"
    return e_fwd, e_adj


# ------------------------------------------------------------------ float64 --
@pytest.mark.parametrize("conv_mode", ["direct", "fft"])
def test_plain_f64_apply(gpu, conv_mode):
    """32x32, 15x15 window, one Lissajous period of 4352 samples, float64."""
    cs = case_from(S.plain_f64(), torch.float64, conv_mode)
    assert cs.plan.conv_mode == conv_mode
    _check_apply(cs, F64_APPLY)


@pytest.mark.parametrize("n,radius,t,conv_mode", [
    (37, 9, 3001, "direct"), (37, 9, 3001, "fft"), (61, 60, 2500, "fft"), (20, 3, 999, "direct")])
def test_ragged_f64_apply(gpu, n, radius, t, conv_mode):
    """Odd grid sizes and windows that do not fill the tiles or the FFT lines."""
    tr = S.lissajous(t, ax=0.85, ay=0.8)
    cs = Case(n, S.h_fwhm2(n) * 1.3, radius, tr.r, tr.v, S.blobs(n, 7), torch.float64, conv_mode)
    _check_apply(cs, F64_APPLY, seed=n)


# ------------------------------------------------------------------ float32 --
@pytest.mark.parametrize("n,radius,t,conv_mode", [
    (37, 7, 3001, "direct"), (37, 7, 3001, "fft"), (128, 31, 53856, "direct"), (128, 31, 53856, "fft"),
    (96, 31, 20000, "direct"), (192, 31, 40000, "fft")])
def test_f32_apply(gpu, n, radius, t, conv_mode):
    tr = S.lissajous(t)
    cs = Case(n, S.h_fwhm2(n), radius, tr.r, tr.v, S.ellipses_and_line(n, 0), torch.float32, conv_mode)
    _check_apply(cs, F32_APPLY, seed=t)


def test_headline_shape_apply(gpu):
    """256x256, 53,856 samples, full-size kernel (R = 255, FFT with M = 512):
    the benchmark's problem shape, as a single-problem plan (column kernels
    in the one-column-per-work-group shape, no problem ranges).  The batched
    pair call the benchmark times is checked in test_gpu_measured.py."""
    cs = case_from(S.headline(), torch.float32)
    assert cs.plan.conv_mode == "fft" and cs.plan.fft_size == 512 and cs.plan.radius == 255
    _check_apply(cs, F32_APPLY, seed=5)


def test_independence_shape_apply(gpu):
    """256x256, perturbed partial trajectory with 2^17 samples, full kernel."""
    cs = case_from(S.independence(), torch.float32)
    _check_apply(cs, F32_APPLY, seed=6)


def test_direct_equals_fft_same_window(gpu):
    P = S.plain_f32()
    a = case_from(P, torch.float32, "direct")
    b = case_from(P, torch.float32, "fft")
    c = a.t(a.c)
    sa, sb = Case.host(a.plan.forward(c)), Case.host(b.plan.forward(c))
    assert rel_l2(sa, sb) <= F32_APPLY
    y = a.t(np.random.default_rng(3).standard_normal((P.n_samples, 2)))
    ca, cb = Case.host(a.plan.adjoint(y)), Case.host(b.plan.adjoint(y))
    assert rel_l2(ca, cb) <= F32_APPLY


def test_adjoint_identity_f32(gpu):
    cs = case_from(S.headline(), torch.float32)
    rng = np.random.default_rng(8)
    x = cs.t(rng.standard_normal((cs.n, cs.n)))
    y = cs.t(rng.standard_normal((cs.plan.n_samples, 2)))
    ax = cs.plan.forward(x)
    aty = cs.plan.adjoint(y)
    lhs = float((ax.double() * y.double()).sum())
    rhs = float((x.double() * aty.double()).sum())
    assert abs(lhs - rhs) <= 1e-6 * max(abs(lhs), abs(rhs))


@pytest.mark.parametrize("conv_mode", ["direct", "fft"])
def test_transpose_is_deterministic(gpu, conv_mode):
    P = S.plain_f32()
    cs = case_from(P, torch.float32, conv_mode)
    y = cs.t(np.random.default_rng(4).standard_normal((P.n_samples, 2)))
    outs = [cs.plan.adjoint(y).clone() for _ in range(3)]
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    c = cs.t(cs.c)
    s0 = cs.plan.forward(c).clone()
    assert torch.equal(cs.plan.forward(c), s0)


# ----------------------------------------------------------------- edge cases --
def test_smallest_grid_and_single_sample(gpu):
    x = S.centres(2)
    r = np.array([[x[0], x[1]], [0.0, 0.0], [x[1], x[1]], [x[1], x[0]], [0.1, -0.2]])
    v = np.array([[1.0, 0.5], [-0.3, 2.0], [0.7, 0.7], [1.0, -1.0], [0.0, 3.0]])
    for mode in ("direct", "fft"):
        cs = Case(2, 0.4, 1, r, v, np.array([[1.0, 2.0], [-0.5, 0.25]]), torch.float64, mode)
        _check_apply(cs, F64_APPLY)
        one = Case(2, 0.4, 1, r[1:2], v[1:2], np.array([[1.0, 2.0], [-0.5, 0.25]]), torch.float64, mode)
        _check_apply(one, F64_APPLY)


def test_all_samples_in_one_cell_and_on_the_hull(gpu):
    """A heavily loaded cell (every sample in one base cell) and samples on the
    outermost cell centres, where the fraction is exactly 0 or 1 (a power-of-two
    grid keeps those centres exact in binary)."""
    n = 32
    x = S.centres(n)
    rng = np.random.default_rng(12)
    t = 5000
    r1 = np.stack([rng.uniform(x[10], x[11], t), rng.uniform(x[5], x[6], t)], 1)
    v1 = rng.standard_normal((t, 2))
    hull = np.array([[x[0], x[0]], [x[-1], x[-1]], [x[0], x[-1]], [x[-1], x[0]], [x[-1], 0.0], [0.0, x[-1]]])
    r = np.vstack([r1, hull])
    v = np.vstack([v1, rng.standard_normal((hull.shape[0], 2))])
    for mode in ("direct", "fft"):
        cs = Case(n, 0.05, 6, r, v, S.blobs(n, 2), torch.float64, mode)
        _check_apply(cs, F64_APPLY, seed=1)


def test_domain_error(gpu):
    n = 16
    x = S.centres(n)
    r = torch.tensor([[0.0, 0.0], [x[-1] + 1e-6, 0.0]], dtype=torch.float64, device="cuda")
    v = torch.ones_like(r)
    with pytest.raises(mpik.MpiError) as ei:
        mpik.Plan(n, 0.1, 3, r, v)
    assert ei.value.status == mpik.MPI_ERR_DOMAIN


def test_workspace_too_small(gpu):
    cs = case_from(S.plain_f64(), torch.float64)
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    c = cs.t(cs.c)
    s = torch.empty((cs.plan.n_samples, 2), dtype=torch.float64, device="cuda")
    rc = cs.plan._L.mpi_forward(cs.plan._h, c.data_ptr(), s.data_ptr(), small.data_ptr(), 256,
                                 torch.cuda.current_stream().cuda_stream)
    assert rc == mpik.MPI_ERR_WORKSPACE


# ----------------------------------------------------------------- iteration --
def _oracle_tau(cs, iters=100):
    return 1.0 / O.power_lambda_max(cs.model, iters=iters)


@pytest.mark.parametrize("use_graph", [False, True])
def test_landweber_f64(gpu, use_graph):
    """50 Landweber iterations from c0 = 0 on noiseless data, float64."""
    P = S.plain_f64()
    cs = case_from(P, torch.float64)
    s = cs.model.forward(cs.c)
    tau = _oracle_tau(cs)
    ref = O.iterate(cs.model, s, np.zeros((P.n, P.n)), tau, P.n_iter)
    c = torch.zeros((P.n, P.n), dtype=torch.float64, device="cuda")
    cs.plan.iterate(cs.t(s), c, P.n_iter, tau, use_graph=use_graph)
    assert rel_l2(Case.host(c), ref) <= 1e-10


def test_denoised_iteration_f32(gpu):
    """128x128, 63x63 window, 20 dB noise, 200 gradient + Gaussian-denoise
    iterations, float32."""
    P = S.plain_f32()
    cs = case_from(P, torch.float32)
    s = S.to_f32(S.add_noise(cs.model.forward(cs.c), P.snr_db, seed=1))
    tau = _oracle_tau(cs)
    ref = O.iterate(cs.model, s, np.zeros((P.n, P.n)), tau, P.n_iter, sigma_px=0.5, radius=2)
    c = torch.zeros((P.n, P.n), dtype=torch.float32, device="cuda")
    cs.plan.iterate(cs.t(s), c, P.n_iter, tau, denoise_sigma_px=0.5, denoise_radius=2, use_graph=True)
    assert rel_l2(Case.host(c), ref) <= 1e-4


def test_iteration_independence_shape_f32(gpu):
    """256x256, 2^17 perturbed partial samples, full kernel: 20 iterations."""
    P = S.independence()
    cs = case_from(P, torch.float32)
    s = S.to_f32(S.add_noise(cs.model.forward(cs.c), P.snr_db, seed=1))
    tau = 0.9 * _oracle_tau(cs, iters=15)
    ref = O.iterate(cs.model, s, np.zeros((P.n, P.n)), tau, 20, sigma_px=0.5, radius=2)
    c = torch.zeros((P.n, P.n), dtype=torch.float32, device="cuda")
    cs.plan.iterate(cs.t(s), c, 20, tau, denoise_sigma_px=0.5, denoise_radius=2)
    assert rel_l2(Case.host(c), ref) <= 1e-4


def test_graph_replay_matches_eager(gpu):
    P = S.plain_f32()
    cs = case_from(P, torch.float32)
    s = cs.t(cs.model.forward(cs.c))
    out = []
    tau = 0.9 * _oracle_tau(cs, iters=10)
    for use_graph in (False, True, True):
        c = torch.zeros((P.n, P.n), dtype=torch.float32, device="cuda")
        cs.plan.iterate(s, c, 7, tau, denoise_sigma_px=0.5, use_graph=use_graph)
        torch.cuda.synchronize()
        out.append(c.clone())
    assert torch.equal(out[0], out[1]) and torch.equal(out[1], out[2])


# ------------------------------------------------------- cosine interpolation --
def _interp_gap(cs):
    """Relative gap between the cosine and the bilinear oracle outputs: the
    parity bar must be far below it for the test to tell the two apart."""
    other = O.Model(cs.n, cs.h, cs.radius, cs.r, cs.v, interp="bilinear")
    return rel_l2(other.forward(cs.c), cs.model.forward(cs.c))


@pytest.mark.parametrize("n,radius,t,conv_mode", [
    (37, 9, 3001, "direct"), (37, 9, 3001, "fft"), (61, 60, 2500, "fft"), (20, 3, 999, "direct")])
def test_cosine_f64_apply(gpu, n, radius, t, conv_mode):
    tr = S.lissajous(t, ax=0.85, ay=0.8)
    cs = Case(n, S.h_fwhm2(n) * 1.3, radius, tr.r, tr.v, S.blobs(n, 7), torch.float64, conv_mode, interp="cosine")
    assert _interp_gap(cs) > 1e4 * F64_APPLY
    _check_apply(cs, F64_APPLY, seed=n)


@pytest.mark.parametrize("n,radius,t,conv_mode", [
    (37, 7, 3001, "direct"), (128, 31, 53856, "direct"), (128, 31, 53856, "fft")])
def test_cosine_f32_apply(gpu, n, radius, t, conv_mode):
    tr = S.lissajous(t)
    cs = Case(n, S.h_fwhm2(n), radius, tr.r, tr.v, S.ellipses_and_line(n, 0), torch.float32, conv_mode,
              interp="cosine")
    assert _interp_gap(cs) > 20 * F32_APPLY
    _check_apply(cs, F32_APPLY, seed=t)


def test_cosine_headline_shape_apply(gpu):
    """256x256, 53,856 samples, full-size kernel, cosine interpolation."""
    cs = case_from(S.headline(), torch.float32, interp="cosine")
    assert cs.plan.conv_mode == "fft" and cs.plan.fft_size == 512 and cs.plan.radius == 255
    assert _interp_gap(cs) > 20 * F32_APPLY
    _check_apply(cs, F32_APPLY, seed=5)


def test_cosine_nodes_and_hull(gpu):
    """Samples on cell centres (weights exactly 0 or 1), edge midpoints
    (weight 1/2) and the hull, float64."""
    n = 32
    x = S.centres(n)
    d = 2.0 / n
    rng = np.random.default_rng(21)
    nodes = np.stack([x[rng.integers(0, n, 300)], x[rng.integers(0, n, 300)]], 1)
    mids = np.stack([x[rng.integers(0, n - 1, 300)] + d / 2, x[rng.integers(0, n, 300)]], 1)
    hull = np.array([[x[0], x[0]], [x[-1], x[-1]], [x[0], x[-1]], [x[-1], x[0]]])
    r = np.vstack([nodes, mids, mids[:, ::-1], hull])
    v = rng.standard_normal(r.shape)
    for mode in ("direct", "fft"):
        cs = Case(n, 0.05, 6, r, v, S.blobs(n, 2), torch.float64, mode, interp="cosine")
        _check_apply(cs, F64_APPLY, seed=2)
        # at these points the two interpolators coincide
        bil = O.Model(n, 0.05, 6, cs.r, cs.v).forward(cs.c)
        assert rel_l2(Case.host(cs.plan.forward(cs.t(cs.c))), bil) <= F64_APPLY


def test_mixed_interpolators_in_one_batch(gpu):
    """The interpolator is chosen per problem: bilinear and cosine problems,
    direct and FFT, share every launch of a batch."""
    shapes = [(24, 5, 3000, "direct", "cosine"), (33, 12, 5000, "fft", "bilinear"), (48, 31, 9000, "fft", "cosine"),
              (40, 9, 4000, "direct", "bilinear")]
    specs, models, cs_ = [], [], []
    for i, (n, R, t, mode, interp) in enumerate(shapes):
        tr = S.lissajous(t, ax=0.85, ay=0.8 + 0.02 * i)
        r, v = (np.asarray(a, dtype=np.float32).astype(np.float64) for a in (tr.r, tr.v))
        h = S.h_fwhm2(n) * (0.9 + 0.05 * i)
        specs.append((n, h, R, torch.tensor(r, dtype=torch.float32, device="cuda"),
                      torch.tensor(v, dtype=torch.float32, device="cuda"), mode, interp))
        models.append(O.Model(n, h, R, r, v, interp=interp))
        cs_.append(np.asarray(S.blobs(n, 30 + i), dtype=np.float32).astype(np.float64))
    batch = mpik.Batch(specs, tune=False)
    c_all = torch.cat([torch.tensor(c, dtype=torch.float32, device="cuda").reshape(-1) for c in cs_])
    s_all = batch.forward(c_all)
    rng = np.random.default_rng(3)
    ys = [np.asarray(rng.standard_normal((sp[3].shape[0], 2)), dtype=np.float32).astype(np.float64) for sp in specs]
    g_all = batch.adjoint(torch.cat([torch.tensor(y, dtype=torch.float32, device="cuda").reshape(-1) for y in ys]))
    torch.cuda.synchronize()
    for b, (M, c, y) in enumerate(zip(models, cs_, ys)):
        s = batch.s_views(s_all)[b].double().cpu().numpy()
        g = batch.c_views(g_all)[b].double().cpu().numpy()
        assert rel_l2(s, M.forward(c)) <= F32_APPLY, b
        assert rel_l2(g, M.adjoint(y)) <= F32_APPLY, b


def test_traj_vjp_needs_a_derivative_plan(gpu):
    tr = S.lissajous(500, ax=0.8, ay=0.8)
    r = torch.tensor(tr.r, dtype=torch.float32, device="cuda")
    v = torch.tensor(tr.v, dtype=torch.float32, device="cuda")
    batch = mpik.Batch([(16, 0.1, 5, r, v, "direct", "cosine")], tune=False)
    x = torch.zeros(256, dtype=torch.float32, device="cuda")
    y = torch.zeros(1000, dtype=torch.float32, device="cuda")
    with pytest.raises(mpik.MpiError) as ei:
        batch.traj_vjp(x, y)
    assert ei.value.status == mpik.MPI_ERR_UNSUPPORTED
