"""Pins of the oracle's cosine interpolator (the core stage's interpolation
scheme, read as per-axis weight w(f) = (1 - cos pi f)/2 on the four
surrounding cell centres) against closed forms, exact reproduction of the
fields the scheme spans, the dense transpose and finite differences taken
without frozen cells (the scheme is C^1, so they hold across cell edges)."""
import numpy as np
import pytest

import oracle as O
from paper_2505_22797_amd import synth as S


def test_weight_closed_forms():
    """cos(pi/4) = sqrt(2)/2, cos(pi/3) = 1/2, cos(pi/2) = 0, ... give exact
    weights; the slope is pi/2 sin(pi f), zero at the nodes."""
    f = np.array([0.0, 0.25, 1 / 3, 0.5, 2 / 3, 0.75, 1.0])
    want = np.array([0.0, (2 - np.sqrt(2)) / 4, 0.25, 0.5, 0.75, (2 + np.sqrt(2)) / 4, 1.0])
    assert np.allclose(O.interp_weight(f, "cosine"), want, rtol=0, atol=1e-15)
    slope = np.array([0.0, np.pi * np.sqrt(2) / 4, np.pi * np.sqrt(3) / 4, np.pi / 2,
                      np.pi * np.sqrt(3) / 4, np.pi * np.sqrt(2) / 4, 0.0])
    assert np.allclose(O.interp_weight_d(f, "cosine"), slope, rtol=0, atol=1e-15)
    assert np.array_equal(O.interp_weight(f, "bilinear"), f)
    with pytest.raises(ValueError):
        O.interp_weight(f, "cubic")


def test_weight_derivative_matches_finite_difference():
    f = np.linspace(-0.3, 1.3, 41)
    e = 1e-6
    fd = (O.interp_weight(f + e, "cosine") - O.interp_weight(f - e, "cosine")) / (2 * e)
    assert np.allclose(O.interp_weight_d(f, "cosine"), fd, rtol=0, atol=1e-9)


def _cos_field(n, coef):
    """Fields a + b cos(pi gx) + c cos(pi gy) + d cos(pi gx) cos(pi gy) in the
    cell-unit coordinate g = (x + 1)/delta - 1/2; inside every cell
    cos(pi g) = +-cos(pi f), so the cosine scheme reproduces them exactly."""
    g = np.arange(n, dtype=np.float64)
    GX, GY = np.meshgrid(np.cos(np.pi * g), np.cos(np.pi * g))
    return np.stack([a + b * GX + c_ * GY + d * GX * GY for a, b, c_, d in coef])


def test_cosine_reproduces_cosine_fields():
    n = 11
    coef = np.array([[0.3, -1.2, 0.5, 2.0], [1.0, 0.25, -0.75, -1.5], [-0.4, 0.9, 1.1, 0.6]])
    G = _cos_field(n, coef)
    x = S.centres(n)
    rng = np.random.default_rng(4)
    r = rng.uniform(x[0], x[-1], (80, 2))
    r = np.vstack([r, [[x[-1], x[-1]], [x[0], x[0]], [x[-1], x[0]], [x[3], x[5]], [x[2], x[9]]]])
    v = rng.standard_normal(r.shape)
    s = O.gather(G, r, v, interp="cosine")
    gx = (r[:, 0] + 1) * n / 2 - 0.5
    gy = (r[:, 1] + 1) * n / 2 - 0.5
    cx, cy = np.cos(np.pi * gx), np.cos(np.pi * gy)
    g = np.stack([a + b * cx + c_ * cy + d * cx * cy for a, b, c_, d in coef])
    ref = np.stack([g[0] * v[:, 0] + g[1] * v[:, 1], g[1] * v[:, 0] + g[2] * v[:, 1]], 1)
    assert np.allclose(s, ref, rtol=0, atol=1e-13)
    # the bilinear scheme does not reproduce them (the pin separates the two)
    assert np.max(np.abs(O.gather(G, r, v) - ref)) > 1e-2


def test_nodes_midpoints_and_cell_centres():
    """Both schemes agree where the fractions are 0, 1/2 or 1: node values,
    edge midpoints (mean of two) and the cell middles (mean of four)."""
    n = 8
    rng = np.random.default_rng(2)
    G = rng.standard_normal((3, n, n))
    x = S.centres(n)
    d = 2.0 / n
    r = np.array([[x[2], x[5]], [x[2] + d / 2, x[5]], [x[2], x[5] + d / 2], [x[2] + d / 2, x[5] + d / 2],
                  [x[-1], x[-1]], [x[0], x[-1]]])
    v = np.tile([[1.0, 0.0]], (r.shape[0], 1))          # s = (G_xx, G_xy)
    s = O.gather(G, r, v, interp="cosine")
    assert np.allclose(s, O.gather(G, r, v), rtol=0, atol=1e-14)
    want = [G[:2, 5, 2], (G[:2, 5, 2] + G[:2, 5, 3]) / 2, (G[:2, 5, 2] + G[:2, 6, 2]) / 2,
            (G[:2, 5, 2] + G[:2, 5, 3] + G[:2, 6, 2] + G[:2, 6, 3]) / 4, G[:2, -1, -1], G[:2, -1, 0]]
    assert np.allclose(s, np.array(want), rtol=0, atol=1e-14)


def test_cosine_dense_transpose_and_adjoint_identity():
    n, t = 6, 40
    tr = S.lissajous(t, ax=0.8, ay=0.8)
    M = O.Model(n, 0.3, 5, tr.r, tr.v, interp="cosine")
    A = np.stack([M.forward(e.reshape(n, n)).ravel() for e in np.eye(n * n)], 1)
    AT = np.stack([M.adjoint(e.reshape(t, 2)).ravel() for e in np.eye(2 * t)], 1)
    assert np.max(np.abs(AT - A.T)) <= 1e-13 * np.max(np.abs(A))
    B = np.stack([O.Model(n, 0.3, 5, tr.r, tr.v).forward(e.reshape(n, n)).ravel() for e in np.eye(n * n)], 1)
    assert np.max(np.abs(A - B)) > 1e-3 * np.max(np.abs(B))
    n, t = 24, 900
    tr = S.lissajous(t, ax=0.8, ay=0.8)
    rng = np.random.default_rng(t)
    M = O.Model(n, 0.07, 9, tr.r, tr.v, interp="cosine")
    xx = rng.standard_normal((n, n))
    y = rng.standard_normal((t, 2))
    a, b = float(np.sum(M.forward(xx) * y)), float(np.sum(xx * M.adjoint(y)))
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_position_derivative_across_cell_edges():
    """Unfrozen central differences match the analytic VJP, also for samples
    a hair before a cell edge where the step crosses it, and vanish at nodes."""
    n = 16
    x = S.centres(n)
    d = 2.0 / n
    rng = np.random.default_rng(5)
    tr = S.lissajous(300, ax=0.85, ay=0.8)
    r = np.vstack([tr.r[:200], [[x[4] + d - 1e-9, x[7] + 0.3 * d], [x[9] + 0.6 * d, x[3] + d - 1e-9],
                                [x[6], x[10]]]])
    v = rng.standard_normal(r.shape)
    h = S.h_fwhm2(n) * 1.5
    c = S.blobs(n, 3)
    y = rng.standard_normal(r.shape)
    g_r, g_v = O.Model(n, h, 6, r, v, interp="cosine").traj_vjp(c, y)
    # each sample's signal depends on its own position only: difference that
    # sample's term alone (no cancellation against the others).  A step across
    # a node meets a jump of the second derivative, so the central difference
    # is first order there: the step is kept small.
    f = lambda rr, vv, k: float(y[k] @ O.Model(n, h, 6, rr, vv, interp="cosine").forward(c)[k])
    scale = np.max(np.abs(g_r)) + 1.0
    e = 1e-8
    for k in (0, 17, 123, 199, 200, 201, 202):
        for a in (0, 1):
            dr = np.zeros_like(r)
            dr[k, a] = e
            fd_r = (f(r + dr, v, k) - f(r - dr, v, k)) / (2 * e)
            fd_v = (f(r, v + dr, k) - f(r, v - dr, k)) / (2 * e)
            assert abs(g_r[k, a] - fd_r) <= 1e-6 * scale, (k, a)
            assert abs(g_v[k, a] - fd_v) <= 1e-7 * (abs(fd_v) + 1.0), (k, a)
    assert np.allclose(g_r[202], 0.0, atol=1e-12)       # a node: zero slope on both axes


def test_bilinear_kink_at_cell_edges():
    """The reason for the frozen-cell convention under bilinear sampling: the
    one-sided slopes differ across an edge; under the cosine scheme they agree."""
    n = 16
    x = S.centres(n)
    d = 2.0 / n
    rng = np.random.default_rng(8)
    G = rng.standard_normal((3, n, n))
    v = np.array([[1.0, 0.0]])
    edge = np.array([[x[5], x[7] + 0.4 * d]])
    e = 1e-5
    slope = {}
    for interp in O.INTERPS:
        s = lambda dx: O.gather(G, edge + [[dx, 0.0]], v, interp=interp)[0, 0]
        slope[interp] = ((s(e) - s(0)) / e, (s(0) - s(-e)) / e)
    left, right = slope["bilinear"]
    assert abs(left - right) > 1e-2
    left, right = slope["cosine"]
    assert abs(left - right) <= 1e-3 * (abs(left) + 1.0)


@pytest.mark.parametrize("sigma", [None, 0.5])
def test_unrolled_gradients_cosine_unfrozen(sigma):
    n = 16
    tr = S.lissajous(600, ax=1.0, ay=1.0)
    rho, nu = tr.r.copy(), tr.v.copy()
    ax, ay = 0.85, 0.8
    h = S.h_fwhm2(n) * 1.5
    c_true = S.blobs(n, 3)
    R = 8
    M = O.Model(n, h, R, rho * [ax, ay], nu * [ax, ay], interp="cosine")
    s = M.forward(c_true) + 0.01 * np.random.default_rng(0).standard_normal((rho.shape[0], 2))
    tau = 0.9 / O.power_lambda_max(M, iters=50)
    c0 = np.zeros((n, n))
    K = 4
    _, g = O.unrolled_gradients(n, h, R, ax, ay, rho, nu, s, c_true, c0, tau, K, sigma_px=sigma,
                                interp="cosine")

    def loss(**kw):
        a = dict(h=h, ax=ax, ay=ay)
        a.update(kw)
        return O.unrolled_gradients(n, a["h"], R, a["ax"], a["ay"], rho, nu, s, c_true, c0, tau, K,
                                    sigma_px=sigma, interp="cosine")[0]

    for name, val in (("h", h), ("ax", ax), ("ay", ay)):
        e = 1e-6 * val
        fd = (loss(**{name: val + e}) - loss(**{name: val - e})) / (2 * e)
        assert abs(g[name] - fd) <= 1e-5 * abs(fd), name
