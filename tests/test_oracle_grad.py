"""Pins of the oracle's derivative functions against float64 central finite
differences of the oracle's own forward maps (the derivatives are written out
by hand; the finite differences only evaluate the operator).

Position derivatives use the frozen-cell convention: every sample keeps its
base cell and the bilinear patch is extended, so a finite difference measures
the derivative inside the patch, which is what the analytic formula states.
"""
import numpy as np
import pytest

import oracle as O
from paper_2505_22797_amd import synth as S


def _problem(n=16, t=600, seed=3):
    tr = S.lissajous(t, ax=1.0, ay=1.0)
    rho, nu = tr.r.copy(), tr.v.copy()
    ax, ay = 0.85, 0.8
    h = S.h_fwhm2(n) * 1.5
    c = S.blobs(n, seed)
    return n, h, rho, nu, ax, ay, c


def test_forward_dh_matches_finite_difference():
    n, h, rho, nu, ax, ay, c = _problem()
    for R in (4, n - 1):
        r, v = rho * [ax, ay], nu * [ax, ay]
        a = O.Model(n, h, R, r, v).forward_dh(c)
        e = 1e-6 * h
        fd = (O.Model(n, h + e, R, r, v).forward(c) - O.Model(n, h - e, R, r, v).forward(c)) / (2 * e)
        assert np.linalg.norm(a - fd) <= 1e-7 * np.linalg.norm(fd)


def test_trajectory_vjp_matches_finite_difference():
    n, h, rho, nu, ax, ay, c = _problem(t=300)
    r, v = rho * [ax, ay], nu * [ax, ay]
    M = O.Model(n, h, 6, r, v)
    frozen = M.cells()
    y = np.random.default_rng(1).standard_normal((r.shape[0], 2))
    g_r, g_v = O.Model(n, h, 6, r, v, frozen=frozen).traj_vjp(c, y)
    f = lambda rr, vv: float(np.sum(y * O.Model(n, h, 6, rr, vv, frozen=frozen).forward(c)))
    # inside a frozen patch the signal is linear in each position coordinate and
    # in the velocity, so a large step is exact and avoids cancellation
    e = 1e-3
    for k in (0, 17, 123, 299):
        for ax_ in (0, 1):
            dr = np.zeros_like(r)
            dr[k, ax_] = e
            fd_r = (f(r + dr, v) - f(r - dr, v)) / (2 * e)
            fd_v = (f(r, v + dr) - f(r, v - dr)) / (2 * e)
            assert abs(g_r[k, ax_] - fd_r) <= 1e-9 * (abs(fd_r) + 1.0)
            assert abs(g_v[k, ax_] - fd_v) <= 1e-9 * (abs(fd_v) + 1.0)


@pytest.mark.parametrize("sigma", [None, 0.5])
def test_unrolled_gradients_match_finite_differences(sigma):
    n, h, rho, nu, ax, ay, c_true = _problem()
    R = 8
    M = O.Model(n, h, R, rho * [ax, ay], nu * [ax, ay])
    s = M.forward(c_true) + 0.01 * np.random.default_rng(0).standard_normal((rho.shape[0], 2))
    tau = 0.9 / O.power_lambda_max(M, iters=50)
    frozen = M.cells()
    c0 = np.zeros((n, n))
    K = 5
    _, g = O.unrolled_gradients(n, h, R, ax, ay, rho, nu, s, c_true, c0, tau, K, sigma_px=sigma, frozen=frozen)

    def loss(**kw):
        a = dict(h=h, ax=ax, ay=ay, c0=c0)
        a.update(kw)
        return O.unrolled_gradients(n, a["h"], R, a["ax"], a["ay"], rho, nu, s, c_true, a["c0"], tau, K,
                                    sigma_px=sigma, frozen=frozen)[0]

    for name, val in (("h", h), ("ax", ax), ("ay", ay)):
        e = 1e-6 * val
        fd = (loss(**{name: val + e}) - loss(**{name: val - e})) / (2 * e)
        assert abs(g[name] - fd) <= 1e-6 * abs(fd), name
    for d in S.unit_directions((n, n), 3, seed=7):
        e = 1e-6
        fd = (loss(c0=c0 + e * d) - loss(c0=c0 - e * d)) / (2 * e)
        assert abs(np.sum(g["c0"] * d) - fd) <= 1e-6 * max(abs(fd), 1e-8)


def test_frozen_cells_only_matter_across_edges():
    """An amplitude step moves the samples that lie close to a cell edge into
    the neighbouring cell (a step of 1e-3 here, large enough that some do):
    the unfrozen model gives exactly those samples a new base cell, while
    the frozen convention keeps every sample's base cell."""
    n, h, rho, nu, ax, ay, _ = _problem(n=32, t=4352)
    step = 1e-3
    g0 = (rho * [ax, ay] + 1.0) / (2.0 / n) - 0.5
    g1 = (rho * [ax * (1 + step), ay] + 1.0) / (2.0 / n) - 0.5
    moved = np.floor(g0[:, 0]) != np.floor(g1[:, 0])
    assert 0 < int(moved.sum()) < moved.size // 10
    M = O.Model(n, h, 5, rho * [ax, ay], nu * [ax, ay])
    ix, jy = M.cells()
    Mu = O.Model(n, h, 5, rho * [ax * (1 + step), ay], nu * [ax * (1 + step), ay])
    assert np.array_equal(Mu.cells()[0] != ix, moved)
    Mf = O.Model(n, h, 5, rho * [ax * (1 + step), ay], nu * [ax * (1 + step), ay], frozen=(ix, jy))
    assert np.array_equal(Mf.cells()[0], ix)
