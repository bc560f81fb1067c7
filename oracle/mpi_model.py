"""Float64 reference implementation of the MPI model operator A and its transpose.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Discretisation used throughout (the paper gives the continuous operator; the
readings below are the ones the GPU library implements too):
  * field of view [-1, 1]^2, N x N cell-centred grid, pitch delta = 2/N,
    centre x_i = -1 + (i + 1/2) delta, arrays c[j, i] with j the y index;
  * the core-operator integral (eq. coreoperator) becomes the Riemann sum
    delta^2 * sum_d K_h(delta d) c[. - d] over integer offsets d with
    |d_x|, |d_y| <= R (square window, zero outside the grid, a linear and not
    a circular convolution); R >= N-1 is the untruncated kernel;
  * the field is interpolated between the four surrounding cell centres and
    contracted with the velocity, s_k = A[c](r_k) v_k (eq. core:formula), the
    constant of proportionality taken as +1.  Two interpolators: bilinear
    (weights f, 1 - f per axis) and the cosine interpolation the paper names
    for its core stage, read as the textbook scheme with per-axis weight
    w(f) = (1 - cos pi f)/2 in place of f (tensor product over the axes);
  * A^T is the exact transpose of that finite linear map.
"""
from __future__ import annotations

from fractions import Fraction
from math import comb

import numpy as np

__all__ = [
    "DomainError", "langevin", "langevin_d1", "langevin_d2",
    "kernel_h", "kernel_h_dh", "trace_kernel_h", "kernel_table", "kernel_table_dh",
    "trace_kernel_table", "effective_radius", "fft_size", "conv_direct", "conv_fft", "conv", "conv_adj",
    "bilinear", "interp_weight", "interp_weight_d", "INTERPS", "CHANNELS", "gather", "velocity_forward_difference", "scatter", "forward", "adjoint", "gauss_weights", "denoise",
    "iterate", "power_lambda_max", "unrolled_gradients", "Model",
]


class DomainError(ValueError):
    """A trajectory sample lies outside the hull of the cell centres."""


# ----------------------------------------------------------------------------
# Langevin function and derivatives (eq. momentum; the printed "cosh" is read
# as coth, the only reading with L(0) = 0, L(inf) = 1 and a finite kernel at 0)
# ----------------------------------------------------------------------------
def _coth_series(nterms: int) -> np.ndarray:
    """a_n with coth z - 1/z = sum_{n>=1} a_n z^(2n-1), a_n = 2^(2n) B_2n / (2n)!.
    Bernoulli numbers from the standard recurrence, in exact rationals."""
    B = [Fraction(1)]
    for m in range(1, 2 * nterms + 1):
        B.append(-sum(comb(m + 1, k) * B[k] for k in range(m)) / (m + 1))
    out = []
    for n in range(1, nterms + 1):
        fact = 1
        for q in range(2, 2 * n + 1):
            fact *= q
        out.append(float(Fraction(2 ** (2 * n)) * B[2 * n] / fact))
    return np.array(out)


_SERIES_CUT = 1.0            # |z| below this: Taylor series (radius of convergence pi)
_A = _coth_series(24)        # term ratio <= (1/pi)^2 ~ 0.1, 24 terms reach 1e-24
_P = 2 * np.arange(1, _A.size + 1) - 1          # powers 2n-1


def _series(z: np.ndarray, deriv: int) -> np.ndarray:
    out = np.zeros_like(z)
    for a, p in zip(_A[::-1], _P[::-1]):        # smallest terms first
        if deriv == 0:
            out += a * z ** p
        elif deriv == 1:
            out += a * p * z ** (p - 1)
        else:
            if p >= 2:
                out += a * p * (p - 1) * z ** (p - 2)
    return out


def _split(z):
    z = np.asarray(z, dtype=np.float64)
    small = np.abs(z) < _SERIES_CUT
    za = np.where(small, 1.0, np.abs(z))        # safe argument for the closed forms
    u = np.exp(-2.0 * za)                        # e^{-2|z|}
    one_m_u = -np.expm1(-2.0 * za)               # 1 - e^{-2|z|}
    return z, small, za, u, one_m_u


def langevin(z):
    """L(z) = coth z - 1/z (odd)."""
    z, small, za, u, omu = _split(z)
    big = np.sign(z) * ((1.0 + u) / omu - 1.0 / za)
    return np.where(small, _series(np.where(small, z, 0.0), 0), big)


def langevin_d1(z):
    """L'(z) = 1/z^2 - 1/sinh^2 z (even), with 1/sinh^2 z = 4u/(1-u)^2, u = e^{-2z}."""
    z, small, za, u, omu = _split(z)
    big = 1.0 / za ** 2 - 4.0 * u / omu ** 2
    return np.where(small, _series(np.where(small, z, 0.0), 1), big)


def langevin_d2(z):
    """L''(z) = 2 cosh z / sinh^3 z - 2/z^3 (odd), with cosh/sinh^3 = 4u(1+u)/(1-u)^3."""
    z, small, za, u, omu = _split(z)
    big = np.sign(z) * (8.0 * u * (1.0 + u) / omu ** 3 - 2.0 / za ** 3)
    return np.where(small, _series(np.where(small, z, 0.0), 2), big)


# ----------------------------------------------------------------------------
# MPI kernel (eq. kernel:matrix), rescaled K_h(y) = K(y/h)/h, trace kernel
# (eq. kernel:trace) and the h-derivative of K_h
# ----------------------------------------------------------------------------
def kernel_h(yx, yy, h):
    """K_h(y) = (1/h)[L'(r) P + (L(r)/r)(I - P)], r = |y|/h, P = y y^T/|y|^2.
    Returns the three distinct entries (xx, xy, yy); K_h(0) = I/(3h)."""
    yx = np.asarray(yx, dtype=np.float64)
    yy = np.asarray(yy, dtype=np.float64)
    q = yx * yx + yy * yy
    zero = q == 0.0
    qs = np.where(zero, 1.0, q)
    r = np.sqrt(qs) / h
    a = langevin_d1(r)                   # radial eigenvalue
    b = langevin(r) / r                  # tangential eigenvalue
    kxx = np.where(zero, 1.0 / 3.0, (a * yx * yx + b * yy * yy) / qs) / h
    kxy = np.where(zero, 0.0, (a - b) * yx * yy / qs) / h
    kyy = np.where(zero, 1.0 / 3.0, (a * yy * yy + b * yx * yx) / qs) / h
    return kxx, kxy, kyy


def kernel_h_dh(yx, yy, h):
    """d K_h / d h = -h^-2 [(L'(r) + r L''(r)) P + L'(r)(I - P)], -I/(3h^2) at 0."""
    yx = np.asarray(yx, dtype=np.float64)
    yy = np.asarray(yy, dtype=np.float64)
    q = yx * yx + yy * yy
    zero = q == 0.0
    qs = np.where(zero, 1.0, q)
    r = np.sqrt(qs) / h
    d1 = langevin_d1(r)
    a = d1 + r * langevin_d2(r)
    b = d1
    s = -1.0 / (h * h)
    kxx = s * np.where(zero, 1.0 / 3.0, (a * yx * yx + b * yy * yy) / qs)
    kxy = s * np.where(zero, 0.0, (a - b) * yx * yy / qs)
    kyy = s * np.where(zero, 1.0 / 3.0, (a * yy * yy + b * yx * yx) / qs)
    return kxx, kxy, kyy


def trace_kernel_h(yx, yy, h, dim: int = 2):
    """kappa_h(y) = (1/h)[L'(r) + (dim - 1) L(r)/r] (eq. kernel:trace); at the
    origin the limit dim/(3h)."""
    q = np.asarray(yx, dtype=np.float64) ** 2 + np.asarray(yy, dtype=np.float64) ** 2
    zero = q == 0.0
    r = np.sqrt(np.where(zero, 1.0, q)) / h
    val = langevin_d1(r) + (dim - 1) * langevin(r) / r
    return np.where(zero, dim / 3.0, val) / h


def _offsets(n: int, radius: int):
    R = effective_radius(n, radius)
    d = np.arange(-R, R + 1)
    DX, DY = np.meshgrid(d, d)          # DX[dy+R, dx+R] = dx
    return R, DX, DY, 2.0 / n


def effective_radius(n: int, radius: int) -> int:
    """Offsets beyond N-1 never meet a non-zero cell, so R is capped there."""
    if radius < 0:
        raise ValueError("radius must be >= 0")
    return min(int(radius), n - 1)


# The selection-field gradient G = diag(gx, gy) (Section "Experiment 2"): the
# kernel is evaluated at G y, K_h(G y), and the velocity that multiplies it is
# -G dr/dt (the caller's).  The isotropic setting of the rest of the paper is
# G = -I, for which K_h(G y) = K_h(y) (K is even); grad=(1, 1) gives the same.
def kernel_table(n: int, h: float, radius: int, grad=(1.0, 1.0)) -> np.ndarray:
    """[3, 2R+1, 2R+1] point samples K_h(G delta (dx, dy)), index [ch, dy+R, dx+R]."""
    R, DX, DY, d = _offsets(n, radius)
    return np.stack(kernel_h(grad[0] * d * DX, grad[1] * d * DY, h))


def kernel_table_dh(n: int, h: float, radius: int, grad=(1.0, 1.0)) -> np.ndarray:
    R, DX, DY, d = _offsets(n, radius)
    return np.stack(kernel_h_dh(grad[0] * d * DX, grad[1] * d * DY, h))


def trace_kernel_table(n: int, h: float, radius: int, grad=(1.0, 1.0)) -> np.ndarray:
    R, DX, DY, d = _offsets(n, radius)
    return trace_kernel_h(grad[0] * d * DX, grad[1] * d * DY, h)


# ----------------------------------------------------------------------------
# discretised core operator: G_ch = delta^2 sum_d K_ch(d) c[. - d] (eq. coreoperator)
# ----------------------------------------------------------------------------
def conv_direct(c: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """out[ch, j, i] = sum_{dy,dx} taps[ch, dy+R, dx+R] c[j-dy, i-dx], zero outside.
    Shifted-slice accumulation; taps may be [2R+1, 2R+1] or [C, 2R+1, 2R+1]."""
    c = np.asarray(c, dtype=np.float64)
    single = taps.ndim == 2
    t = taps[None] if single else taps
    R = (t.shape[-1] - 1) // 2
    n = c.shape[0]
    out = np.zeros((t.shape[0], n, n))
    for dy in range(-R, R + 1):
        if abs(dy) >= n:
            continue
        jd = slice(max(dy, 0), n + min(dy, 0))            # output rows j
        js = slice(max(-dy, 0), n - max(dy, 0))           # source rows j - dy
        for dx in range(-R, R + 1):
            if abs(dx) >= n:
                continue
            id_ = slice(max(dx, 0), n + min(dx, 0))
            is_ = slice(max(-dx, 0), n - max(dx, 0))
            out[:, jd, id_] += t[:, dy + R, dx + R, None, None] * c[None, js, is_]
    return out[0] if single else out


def fft_size(n: int, radius: int) -> int:
    """Smallest power of two M >= N + R: a circular convolution of that size
    reproduces the linear one on the N x N output window."""
    R = effective_radius(n, radius)
    m = 1
    while m < n + R:
        m *= 2
    return m


def conv_fft(c: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """Same operator as conv_direct through numpy.fft on an M x M periodic grid."""
    c = np.asarray(c, dtype=np.float64)
    single = taps.ndim == 2
    t = taps[None] if single else taps
    R = (t.shape[-1] - 1) // 2
    n = c.shape[0]
    m = 1
    while m < n + R:
        m *= 2
    d = np.arange(-R, R + 1) % m
    cp = np.zeros((m, m))
    cp[:n, :n] = c
    C = np.fft.rfft2(cp)
    out = np.empty((t.shape[0], n, n))
    for ch in range(t.shape[0]):
        kp = np.zeros((m, m))
        kp[np.ix_(d, d)] = t[ch]
        out[ch] = np.fft.irfft2(C * np.fft.rfft2(kp), s=(m, m))[:n, :n]
    return out[0] if single else out


def conv(c, taps, method: str = "auto"):
    if method == "auto":
        method = "direct" if (taps.shape[-1] - 1) // 2 <= 7 else "fft"
    return conv_direct(c, taps) if method == "direct" else conv_fft(c, taps)


def conv_adj(g: np.ndarray, taps: np.ndarray, method: str = "auto") -> np.ndarray:
    """Transpose of c -> conv(c, taps) for [3, ...] taps: sum_ch taps_ch (x) g_ch.
    Each kernel channel is even, K(-d) = K(d), so the transpose of a channel's
    convolution is that same convolution."""
    return conv(g, taps, method).sum(axis=0) if taps.ndim == 2 else \
        sum(conv(g[ch], taps[ch], method) for ch in range(taps.shape[0]))


# ----------------------------------------------------------------------------
# sampling along the trajectory and contraction with the velocity
# (eq. core:formula: s(t) = A[rho](r(t)) v(t)); exact transpose
# ----------------------------------------------------------------------------
def bilinear(r: np.ndarray, n: int, frozen=None):
    """Base cell and fractions of every sample.  g = (x+1)/delta - 1/2 is the
    position in cell-centre units; samples need 0 <= g <= N-1 on both axes.
    i0 = min(floor(g), N-2) so that g = N-1 gives the fraction 1.
    frozen = (ix, jy): keep those base cells and extend the bilinear patch
    (fractions may leave [0, 1]) -- the convention under which finite
    differences in the positions equal the derivative inside the patch."""
    r = np.asarray(r, dtype=np.float64)
    g = (r + 1.0) / (2.0 / n) - 0.5
    if frozen is not None:
        ix, jy = frozen
        return ix, jy, g[:, 0] - ix, g[:, 1] - jy
    if not np.all((g >= 0.0) & (g <= n - 1)):
        raise DomainError("trajectory sample outside the hull of the cell centres")
    i0 = np.minimum(np.floor(g), n - 2).astype(np.int64)
    f = g - i0
    return i0[:, 0], i0[:, 1], f[:, 0], f[:, 1]


INTERPS = ("bilinear", "cosine")


def interp_weight(f, interp="bilinear"):
    """Weight of the upper neighbour along one axis at fraction f (the lower
    one gets 1 - w): f for bilinear; (1 - cos pi f)/2 for the cosine scheme,
    which equals the nodes at f = 0, 1, their mean at f = 1/2, and has zero
    slope at the nodes, so the interpolant is C^1 across cell edges."""
    f = np.asarray(f, dtype=np.float64)
    if interp == "bilinear":
        return f
    if interp == "cosine":
        return 0.5 * (1.0 - np.cos(np.pi * f))
    raise ValueError(f"unknown interpolator {interp!r}")


def interp_weight_d(f, interp="bilinear"):
    """d w / d f of `interp_weight`."""
    f = np.asarray(f, dtype=np.float64)
    if interp == "bilinear":
        return np.ones_like(f)
    if interp == "cosine":
        return 0.5 * np.pi * np.sin(np.pi * f)
    raise ValueError(f"unknown interpolator {interp!r}")


def _corners(r, n, frozen=None, interp="bilinear"):
    ix, jy, fx, fy = bilinear(r, n, frozen)
    wx, wy = interp_weight(fx, interp), interp_weight(fy, interp)
    return [((jy, ix), (1 - wx) * (1 - wy)), ((jy, ix + 1), wx * (1 - wy)),
            ((jy + 1, ix), (1 - wx) * wy), ((jy + 1, ix + 1), wx * wy)]


CHANNELS = ("xy", "x")


def gather(G: np.ndarray, r: np.ndarray, v: np.ndarray, frozen=None, interp="bilinear", channels="xy") -> np.ndarray:
    """s_k = G(r_k) v_k with G = [G_xx, G_xy, G_yy] interpolated from the four
    surrounding cell centres.  channels "x": only the x receive channel is
    measured (Section "Experiment 2"): s_x = (G_xx, G_xy) v, and s_y is 0."""
    n = G.shape[-1]
    g = np.zeros((3, r.shape[0]))
    for (j, i), w in _corners(r, n, frozen, interp):
        g += w * G[:, j, i]
    v = np.asarray(v, dtype=np.float64)
    sy = np.zeros(r.shape[0]) if channels == "x" else g[1] * v[:, 0] + g[2] * v[:, 1]
    return np.stack([g[0] * v[:, 0] + g[1] * v[:, 1], sy], 1)


def scatter(y: np.ndarray, r: np.ndarray, v: np.ndarray, n: int, frozen=None, interp="bilinear",
            channels="xy") -> np.ndarray:
    """Transpose of gather: G'_ch(q) = sum_k w_kq p_k,ch with the products
    p = (y_x v_x, y_x v_y + y_y v_x, y_y v_y) (y_y taken as 0 for channels "x")."""
    y = np.array(y, dtype=np.float64)
    if channels == "x":
        y[:, 1] = 0.0
    v = np.asarray(v, dtype=np.float64)
    p = np.stack([y[:, 0] * v[:, 0], y[:, 0] * v[:, 1] + y[:, 1] * v[:, 0], y[:, 1] * v[:, 1]])
    out = np.zeros((3, n * n))
    for (j, i), w in _corners(r, n, frozen, interp):
        for ch in range(3):
            out[ch] += np.bincount(j * n + i, weights=w * p[ch], minlength=n * n)
    return out.reshape(3, n, n)


def velocity_forward_difference(r: np.ndarray, dt: float) -> np.ndarray:
    """v_k = (r_{k+1} - r_k) / dt from the sampled positions (Section
    "Experiment 2"); the last sample repeats the previous difference."""
    r = np.asarray(r, dtype=np.float64)
    v = np.empty_like(r)
    v[:-1] = (r[1:] - r[:-1]) / dt
    v[-1] = v[-2] if r.shape[0] > 1 else 0.0
    return v


def forward(c, r, v, h, radius, method="auto", interp="bilinear"):
    """A c: convolution with delta^2 K_h, then sampling and contraction."""
    n = c.shape[0]
    taps = (2.0 / n) ** 2 * kernel_table(n, h, radius)
    return gather(conv(c, taps, method), r, v, interp=interp)


def adjoint(y, r, v, h, radius, n, method="auto", interp="bilinear"):
    """A^T y: transpose sampling, then the (self-transpose) convolution."""
    taps = (2.0 / n) ** 2 * kernel_table(n, h, radius)
    return conv_adj(scatter(y, r, v, n, interp=interp), taps, method)


# ----------------------------------------------------------------------------
# iteration: gradient step on |Ac - s|^2 followed by a denoiser, the pattern of
# the half-quadratic-splitting loop (eqs. dec:sub:tik, dec:sub:den); the
# Gaussian smoother stands in for the learned denoiser
# ----------------------------------------------------------------------------
def gauss_weights(sigma_px: float, radius: int) -> np.ndarray:
    m = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-m * m / (2.0 * sigma_px * sigma_px))
    return w / w.sum()


def denoise(c: np.ndarray, sigma_px: float, radius: int) -> np.ndarray:
    """Separable Gaussian smoothing, zero padding, rows then columns."""
    w = gauss_weights(sigma_px, radius)
    n = c.shape[0]
    pad = np.zeros((n + 2 * radius, n))
    pad[radius:radius + n] = c
    tmp = sum(w[k] * pad[k:k + n] for k in range(2 * radius + 1))
    pad = np.zeros((n, n + 2 * radius))
    pad[:, radius:radius + n] = tmp
    return sum(w[k] * pad[:, k:k + n] for k in range(2 * radius + 1))


class Model:
    """A and A^T for one problem with the kernel table and sample cells cached.
    frozen = (ix, jy) fixes the base cells (see `bilinear`); interp is
    "bilinear" or "cosine" (see `interp_weight`); grad = (gx, gy) the gradient
    of the kernel table; channels "xy" or "x" (see `gather`)."""

    def __init__(self, n, h, radius, r, v, method="auto", frozen=None, interp="bilinear", grad=(1.0, 1.0),
                 channels="xy"):
        if interp not in INTERPS:
            raise ValueError(f"unknown interpolator {interp!r}")
        if channels not in CHANNELS:
            raise ValueError(f"unknown channels {channels!r}")
        self.n, self.h, self.radius, self.method, self.interp = n, h, radius, method, interp
        self.grad, self.channels = (float(grad[0]), float(grad[1])), channels
        self.r = np.asarray(r, dtype=np.float64)
        self.v = np.asarray(v, dtype=np.float64)
        if frozen is None:
            bilinear(self.r, n)                      # domain check up front
        self.frozen = frozen
        self.taps = (2.0 / n) ** 2 * kernel_table(n, h, radius, self.grad)

    def cells(self):
        ix, jy, _, _ = bilinear(self.r, self.n, self.frozen)
        return ix, jy

    def field(self, c):
        return conv(c, self.taps, self.method)

    def forward(self, c):
        return gather(self.field(c), self.r, self.v, self.frozen, self.interp, self.channels)

    def adjoint(self, y):
        return conv_adj(scatter(y, self.r, self.v, self.n, self.frozen, self.interp, self.channels), self.taps,
                        self.method)

    def normal(self, c):
        return self.adjoint(self.forward(c))

    # ---- derivatives (the VJP building blocks) ----
    def forward_dh(self, x):
        """(dA/dh) x: the sampling of the convolution with delta^2 dK_h/dh."""
        dtaps = (2.0 / self.n) ** 2 * kernel_table_dh(self.n, self.h, self.radius, self.grad)
        return gather(conv(x, dtaps, self.method), self.r, self.v, self.frozen, self.interp, self.channels)

    def traj_vjp(self, x, y):
        """Gradients of <y, A x> with respect to every sample's position r_k and
        velocity v_k, base cells fixed (the derivative inside the interpolation
        patch).  Returns (g_r, g_v), both [T, 2]."""
        n = self.n
        G = self.field(x)
        ix, jy, fx, fy = bilinear(self.r, n, self.frozen)
        wx, wy = interp_weight(fx, self.interp), interp_weight(fy, self.interp)
        g00, g10 = G[:, jy, ix], G[:, jy, ix + 1]
        g01, g11 = G[:, jy + 1, ix], G[:, jy + 1, ix + 1]
        g = (1 - wx) * (1 - wy) * g00 + wx * (1 - wy) * g10 + (1 - wx) * wy * g01 + wx * wy * g11
        # chain rule: d fraction / d position = N/2, d weight / d fraction = w'
        dwx = (n / 2.0) * interp_weight_d(fx, self.interp)
        dwy = (n / 2.0) * interp_weight_d(fy, self.interp)
        dgx = dwx * ((1 - wy) * (g10 - g00) + wy * (g11 - g01))
        dgy = dwy * ((1 - wx) * (g01 - g00) + wx * (g11 - g10))
        y = np.array(y, dtype=np.float64)
        if self.channels == "x":
            y[:, 1] = 0.0
        v = self.v

        def contract(m, a):        # M(m) a with M = [[m0, m1], [m1, m2]]
            return np.stack([m[0] * a[:, 0] + m[1] * a[:, 1], m[1] * a[:, 0] + m[2] * a[:, 1]], 1)

        g_r = np.stack([np.sum(y * contract(dgx, v), 1), np.sum(y * contract(dgy, v), 1)], 1)
        g_v = contract(g, y)
        return g_r, g_v


def iterate(model: Model, s, c0, tau, n_iter, sigma_px=None, radius=2):
    """c <- D(c - tau A^T (A c - s)), D = identity when sigma_px is None."""
    c = np.array(c0, dtype=np.float64)
    for _ in range(n_iter):
        c = c - tau * model.adjoint(model.forward(c) - s)
        if sigma_px is not None:
            c = denoise(c, sigma_px, radius)
    return c


def unrolled_gradients(n, h, radius, ax, ay, rho, nu, s, c_true, c0, tau, n_iter, sigma_px=None, radius_d=2,
                       frozen=None, method="auto", interp="bilinear"):
    """Loss L = |c_K - c_true|^2 after n_iter steps c <- D(c - tau A^T(A c - s))
    with the trajectory r = (ax rho_x, ay rho_y), v = (ax nu_x, ay nu_y), and
    its gradients with respect to c0, h, ax and ay by the reverse recursion:
      u_k = c_k - tau A^T r_k,  r_k = A c_k - s,  c_{k+1} = D u_k;
      gbar_u = D gbar_{c_{k+1}};  gbar_{c_k} = gbar_u - tau A^T A gbar_u;
      dL/dtheta += -tau [ <(dA/dtheta) gbar_u, r_k> + <A gbar_u, (dA/dtheta) c_k> ].
    D is symmetric (an even kernel with zero padding), tau is held fixed."""
    scale = np.array([ax, ay])
    r = np.asarray(rho) * scale
    v = np.asarray(nu) * scale
    M = Model(n, h, radius, r, v, method=method, frozen=frozen, interp=interp)
    D = (lambda x: denoise(x, sigma_px, radius_d)) if sigma_px is not None else (lambda x: x)
    cs, rs = [], []
    c = np.array(c0, dtype=np.float64)
    for _ in range(n_iter):
        res = M.forward(c) - s
        cs.append(c)
        rs.append(res)
        c = D(c - tau * M.adjoint(res))
    loss = float(np.sum((c - c_true) ** 2))
    gbar = 2.0 * (c - c_true)
    gh = gax = gay = 0.0
    for k in reversed(range(n_iter)):
        gu = D(gbar)
        q = M.forward(gu)
        gh += -tau * (np.sum(M.forward_dh(gu) * rs[k]) + np.sum(q * M.forward_dh(cs[k])))
        gr1, gv1 = M.traj_vjp(gu, rs[k])
        gr2, gv2 = M.traj_vjp(cs[k], q)
        gr, gv = gr1 + gr2, gv1 + gv2
        gax += -tau * (np.sum(gr[:, 0] * rho[:, 0]) + np.sum(gv[:, 0] * nu[:, 0]))
        gay += -tau * (np.sum(gr[:, 1] * rho[:, 1]) + np.sum(gv[:, 1] * nu[:, 1]))
        gbar = gu - tau * M.adjoint(q)
    return loss, {"c0": gbar, "h": gh, "ax": gax, "ay": gay}


def power_lambda_max(model: Model, iters: int = 100, seed: int = 0) -> float:
    """Largest eigenvalue of A^T A by power iteration from a seeded start."""
    x = np.random.default_rng(seed).standard_normal((model.n, model.n))
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = model.normal(x)
        lam = float(np.linalg.norm(y))
        x = y / lam
    return lam
