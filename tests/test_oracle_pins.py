"""Pins of the float64 oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: mpmath evaluations of the
paper's definitions (eqs. momentum, kernel:matrix, kernel:trace), the
magnetisation whose Jacobian the kernel is, brute-force dense matrices,
library special cases (numpy.fft, scipy), closed forms and invariants.  The
paper prints no operator values, so none of these pins is a printed value.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.ndimage
import scipy.signal

import oracle as O
from paper_2505_22797_amd import synth as S

mpmath.mp.dps = 40


# --------------------------------------------------------------------------
# mpmath versions of the paper's scalar definitions (independent evaluations)
# --------------------------------------------------------------------------
def mp_L(z):
    z = mpmath.mpf(z)
    return mpmath.coth(z) - 1 / z


def mp_magnetisation(yx, yy, h):
    """Equilibrium magnetisation direction field m(y) = L(|y|/h) y/|y| (eq. momentum
    with the field H = y, unit constants); its Jacobian is K_h."""
    nrm = mpmath.sqrt(yx * yx + yy * yy)
    f = mp_L(nrm / h) / nrm
    return f * yx, f * yy


def mp_jacobian(yx, yy, h):
    yx, yy, h = mpmath.mpf(yx), mpmath.mpf(yy), mpmath.mpf(h)
    jxx = mpmath.diff(lambda a: mp_magnetisation(a, yy, h)[0], yx)
    jxy = mpmath.diff(lambda b: mp_magnetisation(yx, b, h)[0], yy)
    jyx = mpmath.diff(lambda a: mp_magnetisation(a, yy, h)[1], yx)
    jyy = mpmath.diff(lambda b: mp_magnetisation(yx, b, h)[1], yy)
    return jxx, jxy, jyx, jyy


def mp_kappa(r, dim=2):
    """Trace kernel for h = 1 (eq. kernel:trace)."""
    r = mpmath.mpf(r)
    if r == 0:
        return mpmath.mpf(dim) / 3
    L1 = mpmath.diff(mp_L, r)
    return L1 + (dim - 1) * mp_L(r) / r


# --------------------------------------------------------------------------
# P1: Langevin function and derivatives
# --------------------------------------------------------------------------
def test_langevin_against_mpmath():
    z = np.logspace(-8, 3, 200)
    ref0 = np.array([float(mp_L(x)) for x in z])
    ref1 = np.array([float(1 / mpmath.mpf(x) ** 2 - 1 / mpmath.sinh(mpmath.mpf(x)) ** 2) for x in z])
    ref2 = np.array([float(mpmath.diff(mp_L, mpmath.mpf(x), 2)) for x in z])
    for got, ref, tol in ((O.langevin(z), ref0, 1e-14), (O.langevin_d1(z), ref1, 1e-14),
                          (O.langevin_d2(z), ref2, 1e-14)):
        assert np.max(np.abs(got - ref) / np.abs(ref)) <= tol


def test_langevin_parity_and_limits():
    z = np.logspace(-6, 2, 50)
    assert np.allclose(O.langevin(-z), -O.langevin(z), rtol=0, atol=0)
    assert np.array_equal(O.langevin_d1(-z), O.langevin_d1(z))
    assert np.allclose(O.langevin_d2(-z), -O.langevin_d2(z), rtol=0, atol=0)
    assert O.langevin(0.0) == 0.0
    assert abs(O.langevin_d1(0.0) - 1.0 / 3.0) < 1e-16
    assert abs(O.langevin(1e-9) / 1e-9 - 1.0 / 3.0) < 1e-16
    big = np.array([50.0, 200.0, 1000.0])
    assert np.allclose(O.langevin(big), 1.0 - 1.0 / big, rtol=1e-15)
    assert np.allclose(O.langevin_d1(big) * big ** 2, 1.0, rtol=1e-15)
    # the series/closed-form switch is continuous
    e = 1e-12
    for f in (O.langevin, O.langevin_d1, O.langevin_d2):
        assert abs(f(1.0 - e) - f(1.0 + e)) < 1e-11


# --------------------------------------------------------------------------
# P2: the kernel is the Jacobian of the magnetisation, and its structure
# --------------------------------------------------------------------------
@pytest.mark.parametrize("h", [1.0, 0.0213, 0.37])
def test_kernel_is_jacobian_of_magnetisation(h):
    rng = np.random.default_rng(11)
    pts = rng.uniform(-1, 1, (12, 2)) * h * np.array([[0.01], [0.3], [1], [3], [10], [40]] * 2)
    for yx, yy in pts:
        kxx, kxy, kyy = (float(a) for a in O.kernel_h(yx, yy, h))
        jxx, jxy, jyx, jyy = (float(a) for a in mp_jacobian(yx, yy, h))
        scale = abs(jxx) + abs(jyy)
        assert abs(jxy - jyx) <= 1e-20 + 1e-25 * scale
        for got, ref in ((kxx, jxx), (kxy, jxy), (kyy, jyy)):
            assert abs(got - ref) <= 1e-13 * scale


def test_kernel_eigenstructure():
    h = 0.05
    for yx, yy in [(0.01, 0.0), (0.03, 0.04), (-0.2, 0.07), (1e-4, -3e-4)]:
        kxx, kxy, kyy = (float(a) for a in O.kernel_h(yx, yy, h))
        K = np.array([[kxx, kxy], [kxy, kyy]])
        r = math.hypot(yx, yy) / h
        u = np.array([yx, yy]) / math.hypot(yx, yy)
        w = np.array([-u[1], u[0]])
        radial = float(mpmath.diff(mp_L, r)) / h
        tangential = float(mp_L(r) / r) / h
        assert np.allclose(K @ u, radial * u, rtol=0, atol=1e-13 * abs(K).max())
        assert np.allclose(K @ w, tangential * w, rtol=0, atol=1e-13 * abs(K).max())


def test_kernel_origin_scaling_and_symmetries():
    n, h, R = 16, 0.07, 15
    T = O.kernel_table(n, h, R)
    assert T.shape == (3, 2 * R + 1, 2 * R + 1)
    assert T[0, R, R] == pytest.approx(1 / (3 * h), rel=1e-15)
    assert T[2, R, R] == pytest.approx(1 / (3 * h), rel=1e-15)
    assert T[1, R, R] == 0.0
    assert np.allclose(T[0], T[2].T, rtol=1e-15, atol=0)            # K_xx(a,b) = K_yy(b,a)
    assert np.allclose(T[1], -T[1][:, ::-1], rtol=1e-15, atol=0)    # odd in dx
    assert np.allclose(T[1], -T[1][::-1, :], rtol=1e-15, atol=0)    # odd in dy
    assert np.allclose(T[0], T[0][::-1, ::-1], rtol=0, atol=0)      # even
    # K_h(y) = K(y / h) / h
    y = np.array([0.013, -0.4, 2.0])
    a = np.stack(O.kernel_h(y, 0.5 * y, h))
    b = np.stack(O.kernel_h(y / h, 0.5 * y / h, 1.0)) / h
    assert np.allclose(a, b, rtol=1e-14, atol=0)


def test_trace_is_trace_kernel():
    h = 0.03
    rng = np.random.default_rng(5)
    for yx, yy in rng.uniform(-0.3, 0.3, (10, 2)):
        kxx, _, kyy = O.kernel_h(yx, yy, h)
        ref = float(mp_kappa(math.hypot(yx, yy) / h)) / h
        assert abs(kxx + kyy - ref) <= 1e-13 * abs(ref)
        assert abs(O.trace_kernel_h(yx, yy, h) - ref) <= 1e-13 * abs(ref)


def test_kernel_h_derivative():
    """d K_h / d h against mpmath differentiation of the magnetisation Jacobian."""
    for yx, yy, h in [(0.02, 0.01, 0.03), (-0.3, 0.2, 0.11), (1e-3, -2e-3, 0.5)]:
        got = np.array([float(a) for a in O.kernel_h_dh(yx, yy, h)])
        ref = []
        for idx in (0, 1, 3):
            ref.append(float(mpmath.diff(lambda hh: mp_jacobian(yx, yy, hh)[idx], mpmath.mpf(h))))
        ref = np.array(ref)
        assert np.allclose(got, ref, rtol=0, atol=1e-9 * np.abs(ref).max())
    assert O.kernel_h_dh(0.0, 0.0, 0.2)[0] == pytest.approx(-1 / (3 * 0.04), rel=1e-15)


def test_half_maximum_radius_constant():
    """The 2-pixel-FWHM rule: kappa(r*) = kappa(0)/2 for the constant used by
    the input generator, found here by mpmath root finding."""
    root = mpmath.findroot(lambda r: mp_kappa(r) - mp_kappa(0) / 2, 2.9)
    assert abs(float(root) - S.R_HALF) < 1e-13
    n = 128
    h = S.h_fwhm2(n)
    d = 2.0 / n
    assert O.trace_kernel_h(d, 0.0, h) == pytest.approx(O.trace_kernel_h(0.0, 0.0, h) / 2, rel=1e-12)


# --------------------------------------------------------------------------
# P3: the convolution against brute force and numpy.fft
# --------------------------------------------------------------------------
def dense_conv_matrix(n, h, radius):
    """Brute-force N^2 x N^2 matrices (one per channel) from the definition,
    quadruple loop over output and input cells, kernel at delta*(i-i', j-j')."""
    d = 2.0 / n
    R = min(radius, n - 1)
    mats = np.zeros((3, n * n, n * n))
    for j in range(n):
        for i in range(n):
            for jj in range(n):
                for ii in range(n):
                    if abs(i - ii) <= R and abs(j - jj) <= R:
                        k = O.kernel_h(d * (i - ii), d * (j - jj), h)
                        for ch in range(3):
                            mats[ch, j * n + i, jj * n + ii] = d * d * float(k[ch])
    return mats


@pytest.mark.parametrize("n,radius", [(5, 0), (5, 1), (6, 2), (7, 6), (8, 3), (8, 20)])
def test_conv_against_dense_matrix(n, radius):
    h = 0.21
    rng = np.random.default_rng(n * 100 + radius)
    c = rng.standard_normal((n, n))
    mats = dense_conv_matrix(n, h, radius)
    ref = np.stack([mats[ch] @ c.ravel() for ch in range(3)]).reshape(3, n, n)
    taps = (2.0 / n) ** 2 * O.kernel_table(n, h, radius)
    for got in (O.conv_direct(c, taps), O.conv_fft(c, taps)):
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    # each channel matrix is symmetric: the convolution is its own transpose
    for ch in range(3):
        assert np.allclose(mats[ch], mats[ch].T, rtol=0, atol=0)


@pytest.mark.parametrize("n,radius", [(32, 7), (24, 23), (20, 9), (17, 16)])
def test_conv_fft_matches_direct(n, radius):
    rng = np.random.default_rng(radius)
    c = rng.standard_normal((n, n))
    taps = O.kernel_table(n, 0.05, radius)
    a = O.conv_direct(c, taps)
    b = O.conv_fft(c, taps)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_fft_size_is_alias_free():
    assert O.fft_size(256, 255) == 512
    assert O.fft_size(128, 31) == 256
    assert O.fft_size(256, 31) == 512
    assert O.fft_size(64, 31) == 128


# --------------------------------------------------------------------------
# P4: delta phantom and samples on cell centres
# --------------------------------------------------------------------------
def test_delta_phantom_node_samples():
    """With c = e_q / delta^2 the field is the kernel centred on x_q; a sample
    on a cell centre returns that kernel value contracted with the velocity,
    evaluated here from the magnetisation Jacobian in mpmath."""
    n, h, R = 12, 0.15, 11
    d = 2.0 / n
    x = S.centres(n)
    qj, qi = 4, 7
    c = np.zeros((n, n))
    c[qj, qi] = 1.0 / d ** 2
    rng = np.random.default_rng(2)
    pts = [(pj, pi) for pj, pi in rng.integers(0, n, (8, 2))] + [(qj, qi), (n - 1, n - 1), (0, 0)]
    r = np.array([[x[pi], x[pj]] for pj, pi in pts])
    v = rng.standard_normal(r.shape)
    s = O.forward(c, r, v, h, R)
    for k, (pj, pi) in enumerate(pts):
        yx, yy = d * (pi - qi), d * (pj - qj)
        if (yx, yy) == (0.0, 0.0):
            K = np.eye(2) / (3 * h)
        else:
            jxx, jxy, _, jyy = (float(a) for a in mp_jacobian(yx, yy, h))
            K = np.array([[jxx, jxy], [jxy, jyy]])
        assert np.allclose(s[k], K @ v[k], rtol=0, atol=1e-12 * np.abs(K).max() * np.abs(v[k]).max())


def test_delta_phantom_between_nodes():
    """Off the centres the signal is the bilinear blend of the kernel values at
    the four surrounding centres."""
    n, h, R = 10, 0.2, 9
    d = 2.0 / n
    x = S.centres(n)
    qj, qi = 3, 5
    c = np.zeros((n, n))
    c[qj, qi] = 1.0 / d ** 2
    fx, fy = 0.3, 0.85
    r = np.array([[x[2] + fx * d, x[6] + fy * d]])
    v = np.array([[0.7, -1.3]])
    s = O.forward(c, r, v, h, R)
    acc = np.zeros(2)
    for (jj, ii), w in [((6, 2), (1 - fx) * (1 - fy)), ((6, 3), fx * (1 - fy)),
                        ((7, 2), (1 - fx) * fy), ((7, 3), fx * fy)]:
        jxx, jxy, _, jyy = (float(a) for a in mp_jacobian(d * (ii - qi), d * (jj - qj), h))
        acc += w * np.array([[jxx, jxy], [jxy, jyy]]) @ v[0]
    assert np.allclose(s[0], acc, rtol=1e-12)


def test_bilinear_reproduces_bilinear_fields():
    """Interpolating a field that is bilinear in (x, y) is exact anywhere,
    including the last centre (fraction 1) and the first (fraction 0)."""
    n = 9
    x = S.centres(n)
    X, Y = np.meshgrid(x, x)
    coef = np.array([[0.3, -1.2, 0.5, 2.0], [1.0, 0.25, -0.75, -1.5], [-0.4, 0.9, 1.1, 0.6]])
    G = np.stack([a + b * X + c_ * Y + e * X * Y for a, b, c_, e in coef])
    rng = np.random.default_rng(9)
    r = rng.uniform(x[0], x[-1], (50, 2))
    r = np.vstack([r, [[x[-1], x[-1]], [x[0], x[0]], [x[-1], x[0]], [x[3], x[5]]]])
    v = rng.standard_normal(r.shape)
    s = O.gather(G, r, v)
    g = np.stack([a + b * r[:, 0] + c_ * r[:, 1] + e * r[:, 0] * r[:, 1] for a, b, c_, e in coef])
    ref = np.stack([g[0] * v[:, 0] + g[1] * v[:, 1], g[1] * v[:, 0] + g[2] * v[:, 1]], 1)
    assert np.allclose(s, ref, rtol=0, atol=1e-13)


def test_domain_error():
    n = 16
    x = S.centres(n)
    v = np.ones((1, 2))
    O.bilinear(np.array([[x[0], x[-1]]]), n)          # the hull itself is inside
    for bad in ([x[0] - 1e-9, 0.0], [0.0, x[-1] + 1e-9], [1.0, 0.0]):
        with pytest.raises(O.DomainError):
            O.forward(np.zeros((n, n)), np.array([bad]), v, 0.1, 3)


# --------------------------------------------------------------------------
# P5: transpose
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,radius,t", [(6, 5, 40), (32, 7, 4352), (24, 23, 900), (16, 3, 2000)])
def test_adjoint_identity(n, radius, t):
    tr = S.lissajous(t, ax=0.8, ay=0.8)
    rng = np.random.default_rng(t)
    M = O.Model(n, 0.07, radius, tr.r, tr.v)
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((t, 2))
    a = float(np.sum(M.forward(x) * y))
    b = float(np.sum(x * M.adjoint(y)))
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_dense_transpose():
    n, t = 6, 40
    tr = S.lissajous(t, ax=0.8, ay=0.8)
    M = O.Model(n, 0.3, 5, tr.r, tr.v)
    A = np.stack([M.forward(e.reshape(n, n)).ravel() for e in np.eye(n * n)], 1)
    AT = np.stack([M.adjoint(e.reshape(t, 2)).ravel() for e in np.eye(2 * t)], 1)
    assert np.max(np.abs(AT - A.T)) <= 1e-13 * np.max(np.abs(A))


# --------------------------------------------------------------------------
# P6-P8: trace identity, symmetries, linearity
# --------------------------------------------------------------------------
def test_trace_identity_scalar_convolution():
    """G_xx + G_yy equals the scalar convolution with the trace kernel
    (eq. convolution:trace), the latter done by scipy with an mpmath table."""
    n, h, R = 16, 0.09, 15
    d = 2.0 / n
    kap = np.array([[float(mp_kappa(math.hypot(dx, dy) * d / h)) / h for dx in range(-R, R + 1)]
                    for dy in range(-R, R + 1)])
    c = np.random.default_rng(1).uniform(0, 1, (n, n))
    ref = d * d * scipy.signal.convolve2d(c, kap, mode="full")[R:R + n, R:R + n]
    G = O.conv(c, d * d * O.kernel_table(n, h, R), "direct")
    assert np.max(np.abs(G[0] + G[2] - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_axis_swap_and_mirror():
    n, t = 20, 700
    tr = S.lissajous(t)
    c = S.blobs(n, 3)
    h, R = 0.1, 8
    s = O.forward(c, tr.r, tr.v, h, R)
    s_sw = O.forward(c.T, tr.r[:, ::-1], tr.v[:, ::-1], h, R)
    assert np.allclose(s_sw, s[:, ::-1], rtol=1e-13, atol=1e-13 * np.abs(s).max())
    taps = (2.0 / n) ** 2 * O.kernel_table(n, h, R)
    G = O.conv(c, taps)
    Gm = O.conv(c[:, ::-1], taps)
    assert np.allclose(Gm[1], -G[1][:, ::-1], rtol=0, atol=1e-13 * np.abs(G).max())
    assert np.allclose(Gm[0], G[0][:, ::-1], rtol=0, atol=1e-13 * np.abs(G).max())


def test_linearity():
    n, t = 16, 500
    tr = S.lissajous(t)
    rng = np.random.default_rng(4)
    M = O.Model(n, 0.1, 6, tr.r, tr.v)
    a, b = rng.standard_normal((2, n, n))
    assert np.allclose(M.forward(2.5 * a - b), 2.5 * M.forward(a) - M.forward(b), atol=1e-12)
    v2 = rng.standard_normal(tr.v.shape)
    c = S.blobs(n, 1)
    s1 = O.forward(c, tr.r, tr.v, 0.1, 6)
    s2 = O.forward(c, tr.r, v2, 0.1, 6)
    s12 = O.forward(c, tr.r, tr.v - 3 * v2, 0.1, 6)
    assert np.allclose(s12, s1 - 3 * s2, atol=1e-12)


# --------------------------------------------------------------------------
# iteration pieces
# --------------------------------------------------------------------------
def test_denoise_matches_scipy_gaussian():
    c = np.random.default_rng(0).standard_normal((23, 23))
    ref = scipy.ndimage.gaussian_filter(c, 0.5, mode="constant", cval=0.0, truncate=4.0)
    assert np.allclose(O.denoise(c, 0.5, 2), ref, rtol=0, atol=1e-15)
    assert O.gauss_weights(0.5, 2).sum() == pytest.approx(1.0, rel=1e-15)


def test_power_iteration_against_eigvalsh():
    n, t = 6, 60
    tr = S.lissajous(t, ax=0.8, ay=0.8)
    M = O.Model(n, 0.3, 5, tr.r, tr.v)
    A = np.stack([M.forward(e.reshape(n, n)).ravel() for e in np.eye(n * n)], 1)
    lam = np.linalg.eigvalsh(A.T @ A)[-1]
    assert O.power_lambda_max(M, iters=300) == pytest.approx(lam, rel=1e-10)


def test_denoised_iteration_is_the_dense_composition():
    """The denoised iteration (the data step of eq. dec:sub:tik's splitting
    followed by the denoiser, Section "Deconvolution Stage"): c <- D(c - tau
    A^T (A c - s)).  At N = 6 the same recursion is written with dense
    matrices: A from the operator's columns, A^T as its matrix transpose, and
    D from scipy's Gaussian filter (sigma 0.5 px, truncated at 4 sigma, i.e.
    radius 2, zero padding) applied to unit images.  The other composition
    order, c <- D(c) - tau A^T (A D(c) - s), is checked to differ by far more
    than the tolerance, so the pin tells the two apart."""
    n, t = 6, 50
    tr = S.lissajous(t, ax=0.8, ay=0.8)
    M = O.Model(n, 0.3, 5, tr.r, tr.v)
    A = np.stack([M.forward(e.reshape(n, n)).ravel() for e in np.eye(n * n)], 1)
    D = np.stack([scipy.ndimage.gaussian_filter(e.reshape(n, n), 0.5, mode="constant", cval=0.0,
                                                truncate=4.0).ravel() for e in np.eye(n * n)], 1)
    rng = np.random.default_rng(12)
    s = rng.standard_normal((t, 2))
    c0 = rng.uniform(0, 1, (n, n))
    tau = 0.9 / np.linalg.eigvalsh(A.T @ A)[-1]
    K = 7
    x = c0.ravel().copy()
    y = c0.ravel().copy()
    for _ in range(K):
        x = D @ (x - tau * A.T @ (A @ x - s.ravel()))
        y = D @ y
        y = y - tau * A.T @ (A @ y - s.ravel())
    got = O.iterate(M, s, c0, tau, K, sigma_px=0.5, radius=2).ravel()
    assert np.max(np.abs(got - x)) <= 1e-13 * np.max(np.abs(x))
    assert np.max(np.abs(y - x)) >= 1e-3 * np.max(np.abs(x))
    # without the denoiser: the plain Landweber recursion
    z = c0.ravel().copy()
    for _ in range(K):
        z = z - tau * A.T @ (A @ z - s.ravel())
    assert np.max(np.abs(O.iterate(M, s, c0, tau, K).ravel() - z)) <= 1e-13 * np.max(np.abs(z))


def test_landweber_residual_non_increasing():
    P = S.plain_f64()
    r, v = S.to_f32(P.traj.r), S.to_f32(P.traj.v)
    M = O.Model(P.n, P.h, P.radius, r, v)
    s = M.forward(P.c)
    tau = 1.0 / O.power_lambda_max(M)
    c = np.zeros_like(P.c)
    prev = np.linalg.norm(s)
    for _ in range(P.n_iter):
        c = O.iterate(M, s, c, tau, 1)
        res = np.linalg.norm(M.forward(c) - s)
        assert res <= prev * (1 + 1e-12)
        prev = res
    assert prev < 0.5 * np.linalg.norm(s)


# --------------------------------------------------------------------------
# P12: positive semi-definiteness of the sampled kernels (diagnostic)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [8, 12])
def test_sampled_kernels_positive_semidefinite(n):
    h = S.h_fwhm2(n) * 3
    x = S.centres(n)
    X, Y = np.meshgrid(x, x)
    px, py = X.ravel(), Y.ravel()
    DX = px[:, None] - px[None, :]
    DY = py[:, None] - py[None, :]
    kap = O.trace_kernel_h(DX, DY, h)
    ev = np.linalg.eigvalsh(kap)
    assert ev[0] >= -1e-12 * ev[-1]
    kxx, kxy, kyy = O.kernel_h(DX, DY, h)
    big = np.block([[kxx, kxy], [kxy, kyy]])
    ev = np.linalg.eigvalsh(big)
    assert ev[0] >= -1e-12 * ev[-1]


# --------------------------------------------------------------------------
# Table 1 consistency (tests/golden/table1.txt)
# --------------------------------------------------------------------------
def test_table1_trajectory_frequencies():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1.txt")
    vals = {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            vals[k.strip()] = float(v)
    base = vals["base_frequency_hz"]
    npts = vals["sampling_points"]
    assert npts / base == pytest.approx(vals["repetition_time_s"], rel=1e-12)
    cycles = sorted(npts / vals[k] for k in ("divider_x", "divider_y"))
    assert cycles == [16.0, 17.0]
    assert sorted(S.LISSAJOUS_CYCLES) == [16, 17]
    assert S.SAMPLES_PER_PERIOD == int(npts)
    # particle parameters give the saturation field of eq. hsat
    hsat = vals["k_boltzmann"] * vals["temperature_k"] / (
        vals["mu0"] * vals["m_sat"] * math.pi / 6 * vals["core_diameter_m"] ** 3)
    assert vals["mu0"] * hsat * 1e3 == pytest.approx(1.76, abs=5e-3)     # mT


def test_synthetic_workloads_inside_domain():
    for P in (S.plain_f64(), S.plain_f32(), S.headline(), S.independence()):
        O.bilinear(S.to_f32(P.traj.r), P.n)
    for P in S.batch_problems(12):
        O.bilinear(S.to_f32(P.traj.r), P.n)
