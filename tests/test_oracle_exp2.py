"""Pins of the oracle's Experiment-2 inputs (Section "Experiment 2"): the
anisotropic gradient (kernel K_h(G y), velocity -G dr/dt) against the time
derivative of the magnetisation model itself, x-channel-only data, the K_xx
deconvolution kernel and forward-difference velocities."""
import numpy as np
import pytest

import oracle as O
from paper_2505_22797_amd import synth as S


def _magnetisation(y, h):
    """Langevin magnetisation direction field m_h(y) = L(|y|/h) y/|y| (eq.
    momentum), 0 at the origin; y [..., 2]."""
    q = np.sqrt(np.sum(y * y, axis=-1))
    safe = np.where(q == 0.0, 1.0, q)
    return np.where(q[..., None] == 0.0, 0.0, (O.langevin(safe / h) / safe)[..., None] * y)


@pytest.mark.parametrize("grad", [(1.39, -3.16), (-1.0, -1.0), (0.7, 2.2)])
def test_signal_is_the_time_derivative_of_the_magnetisation(grad):
    """s(t) = d/dt sum_x delta^2 c(x) m_h(G (x - r(t))) equals A_G[c](r) v with
    the kernel table at G y and v = -G dr/dt (samples on cell centres, so the
    interpolation is exact; the whole grid in the window)."""
    n, h = 12, 0.21
    G = np.diag(grad)
    x = S.centres(n)
    X, Y = np.meshgrid(x, x)
    pts = np.stack([X, Y], -1)                         # [j, i, 2]
    c = S.blobs(n, 4)
    d2 = (2.0 / n) ** 2
    w = np.array([0.37, -0.81])                        # dr/dt of a straight path
    r0 = np.array([[x[4], x[7]], [x[9], x[2]], [x[6], x[6]]])

    def M(r):
        return np.sum(d2 * c[..., None] * _magnetisation((pts - r) @ G.T, h), axis=(0, 1))

    e = 1e-6
    want = np.stack([(M(r + e * w) - M(r - e * w)) / (2 * e) for r in r0])
    v = np.tile(-G @ w, (r0.shape[0], 1))
    got = O.Model(n, h, n - 1, r0, v, grad=grad).forward(c)
    assert np.allclose(got, want, rtol=1e-7, atol=1e-9 * np.max(np.abs(want)))


def test_gradient_sign_conventions():
    n, h, R = 10, 0.3, 9
    iso = O.kernel_table(n, h, R)
    assert np.array_equal(O.kernel_table(n, h, R, grad=(-1.0, -1.0)), iso)      # K even
    flip = O.kernel_table(n, h, R, grad=(1.0, -1.0))
    assert np.array_equal(flip[0], iso[0]) and np.array_equal(flip[2], iso[2])
    assert np.allclose(flip[1], -iso[1], atol=0)                                  # K_xy odd in y
    t = O.trace_kernel_table(n, h, R, grad=(1.39, -3.16))
    k = O.kernel_table(n, h, R, grad=(1.39, -3.16))
    assert np.allclose(t, k[0] + k[2], rtol=1e-12)


def test_x_channel_operator_and_transpose():
    n, t = 6, 40
    tr = S.lissajous(t, ax=0.8, ay=0.8)
    full = O.Model(n, 0.3, 5, tr.r, tr.v, interp="cosine")
    xonly = O.Model(n, 0.3, 5, tr.r, tr.v, interp="cosine", channels="x")
    c = S.blobs(n, 1)
    s = xonly.forward(c)
    assert np.array_equal(s[:, 0], full.forward(c)[:, 0]) and not np.any(s[:, 1])
    A = np.stack([xonly.forward(e.reshape(n, n)).ravel() for e in np.eye(n * n)], 1)
    AT = np.stack([xonly.adjoint(e.reshape(t, 2)).ravel() for e in np.eye(2 * t)], 1)
    assert np.max(np.abs(AT - A.T)) <= 1e-13 * np.max(np.abs(A))


def test_x_channel_core_stage():
    """The normal operator stays half the gradient of the x-only objective, and
    the yy channel, which no data reaches, stays 0."""
    n, t, gamma = 8, 300, 3e-4
    rng = np.random.default_rng(1)
    x = S.centres(n)
    r = rng.uniform(x[0], x[-1], (t, 2))
    v = rng.standard_normal((t, 2))
    s = rng.standard_normal((t, 2))
    a = rng.standard_normal((3, n, n))
    g = O.core_normal(a, r, v, gamma, channels="x") - O.core_rhs(s, r, v, n, channels="x")
    d = rng.standard_normal((3, n, n))
    e = 1e-6
    fd = (O.core_objective(a + e * d, s, r, v, gamma, channels="x")
          - O.core_objective(a - e * d, s, r, v, gamma, channels="x")) / (2 * e)
    assert abs(fd - 2 * np.sum(g * d)) <= 1e-7 * abs(fd)
    field, _ = O.core_stage(s, r, v, n, gamma, tol=1e-8, max_iter=3000, channels="x")
    assert not np.any(field[2]) and np.any(field[0]) and np.any(field[1])


def test_xx_deconvolution_kernel():
    n, h, R = 16, 0.1, 15
    k = O.kernel_table(n, h, R, grad=(1.39, -3.16))
    assert np.array_equal(O.trace_taps(n, h, R, "xx", (1.39, -3.16)), (2.0 / n) ** 2 * k[0])
    rho = S.blobs(n, 2)
    u = O.trace_conv(rho, h, R, which="xx", grad=(1.39, -3.16))
    out, info = O.zeroshot_pnp(u, h, R, 2, 1e-3, tol=1e-4, which="xx", grad=(1.39, -3.16))
    assert np.linalg.norm(out - rho) < np.linalg.norm(u / np.max(np.abs(u)) * np.max(rho) - rho)


def test_forward_difference_velocities():
    """Exact on straight paths; on the Experiment-2 figure the forward
    difference is the derivative at the interval midpoint to second order."""
    t = np.linspace(0.0, 1.0, 2001)
    dt = t[1] - t[0]
    r = np.stack([0.3 + 0.5 * t, -0.2 - 0.7 * t], 1)
    assert np.allclose(O.velocity_forward_difference(r, dt), [0.5, -0.7], rtol=1e-12)
    fx, fe, ax, ae, ay = 3.0, 40.0, 0.6, 0.05, 0.7
    pos = lambda tt: np.stack([ax * np.sin(2 * np.pi * fx * tt) + ae * np.sin(2 * np.pi * fe * tt),
                               ay * np.sin(2 * np.pi * fx * tt)], 1)
    vel = lambda tt: np.stack([2 * np.pi * (ax * fx * np.cos(2 * np.pi * fx * tt) + ae * fe * np.cos(2 * np.pi * fe * tt)),
                               2 * np.pi * ay * fx * np.cos(2 * np.pi * fx * tt)], 1)
    v = O.velocity_forward_difference(pos(t), dt)
    mid = vel(t[:-1] + dt / 2)
    scale = (2 * np.pi) ** 3 * (ax * fx ** 3 + ae * fe ** 3)
    assert np.max(np.abs(v[:-1] - mid)) <= scale * dt * dt / 24 * 1.01
    assert np.array_equal(v[-1], v[-2])
