"""Pins of the oracle's Deconvolution Stage (trace convolution, conjugate
gradients, percentile trimming, noise estimate, ZeroShot-PnP schedule) against
dense linear algebra, closed forms, textbook properties of conjugate gradients
and hand-worked examples."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2505_22797_amd import synth as S


def _dense(apply, n):
    return np.stack([apply(e.reshape(n, n)).ravel() for e in np.eye(n * n)], 1)


@pytest.mark.parametrize("n,radius", [(6, 5), (7, 2), (8, 7)])
def test_trace_conv_is_the_trace_of_the_field(n, radius):
    """C_h x equals G_xx + G_yy of the operator's field (eq. convolution:trace)
    and is symmetric (kappa even)."""
    h = 0.3
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n))
    taps = (2.0 / n) ** 2 * O.kernel_table(n, h, radius)
    G = O.conv(x, taps, "direct")
    for method in ("direct", "fft"):
        assert np.allclose(O.trace_conv(x, h, radius, method), G[0] + G[2], rtol=0, atol=1e-13)
    C = _dense(lambda e: O.trace_conv(e, h, radius, "direct"), n)
    assert np.max(np.abs(C - C.T)) <= 1e-14 * np.max(np.abs(C))


def test_cg_solves_the_tikhonov_normal_equations():
    n, R, h, nu = 6, 5, 0.25, 1e-3
    C = _dense(lambda e: O.trace_conv(e, h, R, "direct"), n)
    A = C.T @ C + nu * np.eye(n * n)
    b = np.random.default_rng(1).standard_normal(n * n)
    x, steps, norms = O.cg(lambda v: (A @ v.ravel()).reshape(v.shape), b.reshape(n, n), 1e-13, 500)
    assert np.allclose(x.ravel(), np.linalg.solve(A, b), rtol=0, atol=1e-9 * np.max(np.abs(x)))
    assert norms[-1] <= 1e-13 * norms[0] < norms[-2]


def test_cg_terminates_in_as_many_steps_as_distinct_eigenvalues():
    """In exact arithmetic CG needs at most as many steps as the matrix has
    distinct eigenvalues; four well-separated values here."""
    rng = np.random.default_rng(2)
    lam = np.repeat([1.0, 2.0, 5.0, 9.0], 10)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    A = (Q * lam) @ Q.T
    b = rng.standard_normal(40)
    x, steps, norms = O.cg(lambda v: A @ v, b, 1e-10, 100)
    assert steps == 4
    assert np.allclose(A @ x, b, atol=1e-10)


def test_cg_stop_rule_and_degenerate_inputs():
    A = np.diag(np.linspace(1.0, 50.0, 30))
    b = np.random.default_rng(3).standard_normal(30)
    x, steps, norms = O.cg(lambda v: A @ v, b, 1e-3, 100)
    assert norms[steps] <= 1e-3 * norms[0] < norms[steps - 1]      # the first step that meets the tolerance
    x2, steps2, _ = O.cg(lambda v: A @ v, b, 0.0, steps)            # tol 0: exactly max_iter steps
    assert steps2 == steps and np.array_equal(x2, x)
    x0, s0, _ = O.cg(lambda v: A @ v, np.zeros(30), 1e-3, 100)     # b = 0: no step, x = 0
    assert s0 == 0 and not np.any(x0)
    x0, s0, _ = O.cg(lambda v: A @ v, b, 1e-3, 0)                  # no step allowed
    assert s0 == 0 and not np.any(x0)
    # a multiple of the identity: one step reaches the solution b / (1 + nu)
    x1, s1, _ = O.cg(lambda v: 1.25 * v, b, 1e-12, 10)
    assert s1 == 1 and np.allclose(x1, b / 1.25, rtol=1e-15, atol=0)


def test_percentile_hand_examples():
    assert O.percentile(np.arange(1.0, 22.0), 5) == pytest.approx(2.0, abs=1e-15)       # pos 1.0
    assert O.percentile(np.array([50.0, 10.0, 40.0, 20.0, 30.0]), 5) == pytest.approx(12.0, abs=1e-14)
    assert O.percentile(np.array([3.0, 1.0, 2.0]), 50) == 2.0
    assert O.percentile(np.array([7.0]), 5) == 7.0
    assert O.percentile(np.array([4.0, -1.0]), 0) == -1.0 and O.percentile(np.array([4.0, -1.0]), 100) == 4.0
    x = np.random.default_rng(4).standard_normal((33, 33))
    assert O.percentile(x, 5) == pytest.approx(np.percentile(x, 5), abs=1e-15)      # the library's linear rule
    y, q = O.percentile_clamp(x, 5)
    assert np.all(y >= q) and np.array_equal(y[x >= q], x[x >= q]) and np.all(y[x < q] == q)
    assert np.sum(x < q) == math.ceil(0.05 * (x.size - 1))


def test_noise_sigma_closed_form():
    n = 1000
    assert O.noise_sigma(np.arange(1.0, n + 1.0)) == pytest.approx(math.sqrt((n * n - 1) / 12.0), rel=1e-14)
    assert O.noise_sigma(np.full((9, 9), 3.5)) == 0.0


def _workload(n=24, R=23, seed=0):
    h = S.h_fwhm2(n)
    rho = S.blobs(n, seed)
    u = O.trace_conv(rho, h, R)
    u = u + 0.01 * np.linalg.norm(u) / n * np.random.default_rng(seed).standard_normal(u.shape)
    return n, R, h, rho, u


def test_pnp_first_pass_is_the_tikhonov_solution_and_nu_schedule():
    """With the identity denoiser and no trimming, pass 0 returns the exact
    Tikhonov solution (C^T C + nu0 I)^-1 C^T u, nu_1 equals nu0 (lambda is
    nu0 sigma_1^2), and later nu follow lambda / sigma^2."""
    n, R, h, rho, u = _workload(n=10, R=9)
    nu0 = 1e-4
    out, info = O.zeroshot_pnp(u, h, R, 0, nu0, tol=1e-14, max_iter=5000, clip_pct=None, sigma_px=None)
    C = _dense(lambda e: O.trace_conv(e, h, R), n)
    ref = np.linalg.solve(C.T @ C + nu0 * np.eye(n * n), C.T @ u.ravel()).reshape(n, n)
    assert np.allclose(out, ref, rtol=0, atol=1e-8 * np.max(np.abs(ref)))
    assert info["lam"] == pytest.approx(nu0 * info["sigma"][0] ** 2, rel=1e-15)
    out, info = O.zeroshot_pnp(u, h, R, 3, nu0, tol=1e-6, max_iter=5000, clip_pct=5.0, sigma_px=0.5)
    assert info["nu"][0] == nu0 and len(info["nu"]) == 4
    assert info["nu"][1] == pytest.approx(nu0, rel=1e-15)
    for k in range(1, 4):
        assert info["nu"][k] == pytest.approx(info["lam"] / info["sigma"][k - 1] ** 2, rel=1e-15)


def test_pnp_passes_are_consistent_with_their_parts():
    """Two passes rebuilt from the parts: CG on the pass's normal equations,
    trimming, noise estimate and the Gaussian step."""
    n, R, h, rho, u = _workload(n=16, R=15, seed=1)
    nu0, tol = 1e-3, 1e-4
    out, info = O.zeroshot_pnp(u, h, R, 1, nu0, tol=tol, max_iter=2000, clip_pct=5.0, sigma_px=0.5)
    Cf = lambda x: O.trace_conv(x, h, R)
    rho2 = np.zeros((n, n))
    nu = nu0
    for k in range(2):
        rho1, steps, _ = O.cg(lambda x: Cf(Cf(x)) + nu * x, Cf(u) + nu * rho2, tol, 2000)
        rho1 = np.maximum(rho1, np.percentile(rho1, 5))
        sigma = float(np.std(rho1))
        assert steps == info["cg_steps"][k] and sigma == pytest.approx(info["sigma"][k], rel=1e-12)
        lam = nu0 * sigma ** 2 if k == 0 else lam
        rho2 = O.denoise(rho1, 0.5, 2)
        nu = lam / sigma ** 2
    assert np.allclose(out, rho2, rtol=0, atol=1e-12 * np.max(np.abs(rho2)))


def test_pnp_improves_on_the_trace_image():
    n, R, h, rho, u = _workload(n=32, R=31, seed=2)
    out, info = O.zeroshot_pnp(u, h, R, 3, 1e-4, tol=1e-3, max_iter=2000)
    err = lambda x: np.linalg.norm(x - rho) / np.linalg.norm(rho)
    scale = np.sum(u * rho) / np.sum(u * u)          # best multiple of u
    assert err(out) < 0.5 * err(scale * u)
    assert all(s > 0 for s in info["cg_steps"])
