"""Pins of the oracle's Core Stage (eq. first:step): the graph Laplacian
against closed forms and an explicit loop, the normal operator against finite
differences of the objective written out from the functional, symmetry and
definiteness, exact recovery of a field from noise-free overdetermined data,
and the stationarity of the solution."""
import numpy as np
import pytest

import oracle as O
from paper_2505_22797_amd import synth as S


def _lap_loops(a):
    """The graph Laplacian by explicit loops over cells and their neighbours."""
    n = a.shape[-1]
    out = np.zeros_like(a)
    for j in range(n):
        for i in range(n):
            for dj, di in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                jj, ii = j + dj, i + di
                if 0 <= jj < n and 0 <= ii < n:
                    out[..., j, i] += a[..., jj, ii] - a[..., j, i]
    return out * (n / 2.0) ** 2


def test_laplacian_closed_forms_and_loops():
    n = 9
    x = S.centres(n)
    X, Y = np.meshgrid(x, x)
    lap = O.laplacian(X ** 2 + Y ** 2)
    assert np.allclose(lap[1:-1, 1:-1], 4.0, rtol=0, atol=1e-10)        # 2 per axis in the interior
    assert np.allclose(O.laplacian(np.full((3, n, n), 2.5)), 0.0, atol=1e-12)
    a = np.random.default_rng(0).standard_normal((3, n, n))
    assert np.allclose(O.laplacian(a), _lap_loops(a), rtol=0, atol=1e-10)
    assert abs(np.sum(O.laplacian(a[0]))) <= 1e-9 * np.sum(np.abs(O.laplacian(a[0])))   # sums to zero
    D = np.stack([O.laplacian(e.reshape(5, 5)).ravel() for e in np.eye(25)], 1)
    assert np.allclose(D, D.T, atol=1e-12)
    assert np.max(np.linalg.eigvalsh(D)) <= 1e-9


def _samples(n, t, seed):
    rng = np.random.default_rng(seed)
    x = S.centres(n)
    r = rng.uniform(x[0], x[-1], (t, 2))
    v = rng.standard_normal((t, 2))
    return r, v


@pytest.mark.parametrize("interp", ["cosine", "bilinear"])
def test_normal_operator_is_half_the_objective_gradient(interp):
    """d/de J(a + e d) = 2 <E a - b, d> for the objective of eq. first:step
    written out directly (data term over L, weights 1, 2, 1, delta^2)."""
    n, t, gamma = 8, 300, 3e-4
    r, v = _samples(n, t, 1)
    rng = np.random.default_rng(2)
    s = rng.standard_normal((t, 2))
    a = rng.standard_normal((3, n, n))
    b = O.core_rhs(s, r, v, n, interp)
    g = O.core_normal(a, r, v, gamma, interp) - b
    for k in range(3):
        d = rng.standard_normal((3, n, n))
        e = 1e-6
        fd = (O.core_objective(a + e * d, s, r, v, gamma, interp)
              - O.core_objective(a - e * d, s, r, v, gamma, interp)) / (2 * e)
        assert abs(fd - 2 * np.sum(g * d)) <= 1e-7 * abs(fd), k


def test_normal_operator_symmetric_positive_definite():
    n, t, gamma = 4, 60, 1e-3
    r, v = _samples(n, t, 3)
    E = np.stack([O.core_normal(e.reshape(3, n, n), r, v, gamma).ravel() for e in np.eye(3 * n * n)], 1)
    assert np.max(np.abs(E - E.T)) <= 1e-13 * np.max(np.abs(E))
    assert np.min(np.linalg.eigvalsh(E)) > 0


def test_recovers_a_field_from_overdetermined_noise_free_data():
    n = 8
    t = 30 * 3 * n * n
    r, v = _samples(n, t, 4)
    a_true = np.random.default_rng(5).standard_normal((3, n, n))
    s = O.gather(a_true, r, v, interp="cosine")
    a, steps = O.core_stage(s, r, v, n, gamma=1e-14, tol=1e-12, max_iter=5000)
    assert np.max(np.abs(a - a_true)) <= 1e-6 * np.max(np.abs(a_true)), steps


def test_solution_is_stationary():
    """At the CG solution the objective's directional derivatives vanish
    (relative to those at a = 0)."""
    n, t, gamma = 10, 400, 1e-4
    r, v = _samples(n, t, 6)
    s = np.random.default_rng(7).standard_normal((t, 2))
    a, _ = O.core_stage(s, r, v, n, gamma, tol=1e-11, max_iter=5000)
    rng = np.random.default_rng(8)
    for _ in range(3):
        d = rng.standard_normal((3, n, n))
        e = 1e-5
        J = lambda x: O.core_objective(x, s, r, v, gamma)
        g_sol = (J(a + e * d) - J(a - e * d)) / (2 * e)
        g_zero = (J(e * d) - J(-e * d)) / (2 * e)
        assert abs(g_sol) <= 1e-6 * abs(g_zero)
