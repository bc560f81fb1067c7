"""Float64 reference of the Core Stage: the variational reconstruction of the
matrix-valued core-operator field from the data (s_k, r_k, v_k) (Section "MPI
Core Stage", eq. first:step).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (the paper names the functional, the regulariser and the solver):
  * The unknown is the symmetric field A = [A_xx, A_xy, A_yy] on the N x N
    cell-centred grid.  The interpolator I is the operator's sampling (the
    cosine scheme by default, as the paper uses), contracted with the velocity:
    (I a)_k = M(a(r_k)) v_k; its transpose is the operator's transpose sampling.
  * The regulariser is the squared L2 norm of the Laplacian of the matrix
    field, R_C = integral of |Delta A|_F^2: the Frobenius norm counts the
    off-diagonal entry twice (channel weights 1, 2, 1), and the integral is a
    sum over cells times delta^2.
  * Delta is the 5-point graph Laplacian with spacing delta = 2/N: the sum over
    the in-grid neighbours q of p of (a_q - a_p) / delta^2 (no values outside
    the field of view are assumed; constants are not penalised).  It is
    symmetric, so the Euler-Lagrange equations of eq. first:step read
        (1/L) I^T I a + gamma delta^2 W Delta Delta a = (1/L) I^T s,
    with W = diag(1, 2, 1) over the channels, L the number of samples.
  * They are solved by the conjugate gradients of the Deconvolution Stage's
    oracle (from a = 0, relative residual tolerance, step cap).
  * With only the x receive channel (channels "x", Section "Experiment 2")
    the data term has s_x alone; A_yy then only meets the regulariser and
    stays 0 from a = 0.
"""
from __future__ import annotations

import numpy as np

from .deconv import cg
from .mpi_model import gather, scatter

__all__ = ["laplacian", "core_objective", "core_normal", "core_rhs", "core_stage", "CHANNEL_WEIGHTS"]

CHANNEL_WEIGHTS = np.array([1.0, 2.0, 1.0])     # Frobenius norm of [[xx, xy], [xy, yy]]


def laplacian(a: np.ndarray) -> np.ndarray:
    """Graph Laplacian of every channel of a ([..., N, N]): for each cell, the
    sum over its in-grid 4-neighbours of (neighbour - cell), over delta^2."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[-1]
    out = np.zeros_like(a)
    out[..., 1:, :] += a[..., :-1, :] - a[..., 1:, :]
    out[..., :-1, :] += a[..., 1:, :] - a[..., :-1, :]
    out[..., :, 1:] += a[..., :, :-1] - a[..., :, 1:]
    out[..., :, :-1] += a[..., :, 1:] - a[..., :, :-1]
    return out * (n / 2.0) ** 2


def core_objective(a, s, r, v, gamma, interp="cosine", channels="xy") -> float:
    """(1/L) sum_k |s_k - M(a(r_k)) v_k|^2 + gamma * delta^2 * sum |Delta a|_F^2
    (eq. first:step, discretised as above)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[-1]
    s = np.array(s, dtype=np.float64)
    if channels == "x":
        s[:, 1] = 0.0
    res = s - gather(a, r, v, interp=interp, channels=channels)
    lap = laplacian(a)
    reg = (2.0 / n) ** 2 * float(np.sum(CHANNEL_WEIGHTS[:, None, None] * lap * lap))
    return float(np.sum(res * res)) / res.shape[0] + gamma * reg


def core_normal(a, r, v, gamma, interp="cosine", channels="xy") -> np.ndarray:
    """(1/L) I^T I a + gamma delta^2 W Delta Delta a."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[-1]
    L = np.asarray(r).shape[0]
    data = scatter(gather(a, r, v, interp=interp, channels=channels), r, v, n, interp=interp, channels=channels) / L
    return data + gamma * (2.0 / n) ** 2 * CHANNEL_WEIGHTS[:, None, None] * laplacian(laplacian(a))


def core_rhs(s, r, v, n, interp="cosine", channels="xy") -> np.ndarray:
    """(1/L) I^T s."""
    return scatter(s, r, v, n, interp=interp, channels=channels) / np.asarray(r).shape[0]


def core_stage(s, r, v, n, gamma, tol=1e-3, max_iter=10000, interp="cosine", channels="xy"):
    """The field minimising eq. first:step by CG on its Euler-Lagrange
    equations from a = 0.  Returns (field [3, N, N], CG steps)."""
    b = core_rhs(s, r, v, n, interp, channels)
    a, steps, _ = cg(lambda x: core_normal(x, r, v, gamma, interp, channels), b, tol, max_iter)
    return a, steps
