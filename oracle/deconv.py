"""Float64 reference of the Deconvolution Stage: the scalar trace-kernel
convolution C_h and the ZeroShot-PnP loop around it (Section "Deconvolution
Stage", Algorithm "ZeroShot-PnP", Section "Denoiser Artifact Reduction").

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (the paper gives the loop, not every detail):
  * C_h is the convolution with delta^2 kappa_h, the trace of the kernel
    (eq. kernel:trace), on the same grid, window and quadrature as the
    operator; the trace of the core operator is C_h rho (eq.
    convolution:trace).  kappa_h is even, so C_h^T = C_h.
  * The Tikhonov sub-step (eq. dec:sub:tik) is solved on its normal equations
    (C^T C + nu I) rho_1 = C^T u + nu rho_2 by textbook conjugate gradients
    started from rho_1 = 0; it stops once the recursively updated residual r
    meets |r| <= tol |b| (tested before every step), or after max_iter steps.
  * Trimming (Section "Denoiser Artifact Reduction"): right after the solve,
    values of rho_1 below its p-th percentile (linear interpolation between
    order statistics) are raised to that percentile; the trimmed rho_1 feeds
    the noise estimate and the denoiser.
  * Noise estimate sigma = sqrt of the population variance of rho_1 over the
    pixels.  lambda = nu_0 sigma^2 with the first estimate; then
    nu_{k+1} = lambda / sigma_{k+1}^2 (nu unchanged if sigma = 0).
  * "while k <= n_it" makes n_it + 1 passes, k = 0..n_it; the result is rho_2
    after the last pass.
  * The learned denoiser is replaced by the separable Gaussian of the
    iteration (its noise-level argument has no role in the stand-in); None
    means the identity.
  * With only the x receive channel (Section "Experiment 2") the trace is not
    available and the first diagonal entry is deconvolved with the first
    diagonal entry of the kernel: `which="xx"` uses delta^2 K_xx in place of
    delta^2 kappa_h.  `grad` is the kernel's gradient as in the operator.
"""
from __future__ import annotations

import math

import numpy as np

from .mpi_model import conv, denoise, kernel_table, trace_kernel_table

__all__ = ["trace_taps", "trace_conv", "cg", "percentile", "percentile_clamp", "noise_sigma", "zeroshot_pnp"]


def trace_taps(n: int, h: float, radius: int, which: str = "trace", grad=(1.0, 1.0)) -> np.ndarray:
    """delta^2 kappa_h (which "trace") or delta^2 K_h,xx (which "xx") at the
    integer offsets of the window, [2R+1, 2R+1]."""
    if which == "trace":
        return (2.0 / n) ** 2 * trace_kernel_table(n, h, radius, grad)
    if which == "xx":
        return (2.0 / n) ** 2 * kernel_table(n, h, radius, grad)[0]
    raise ValueError(f"unknown deconvolution kernel {which!r}")


def trace_conv(x: np.ndarray, h: float, radius: int, method: str = "auto", which: str = "trace",
               grad=(1.0, 1.0)) -> np.ndarray:
    """C_h x (eq. convolution:trace): zero outside the grid, linear convolution."""
    x = np.asarray(x, dtype=np.float64)
    return conv(x, trace_taps(x.shape[0], h, radius, which, grad), method)


def cg(apply, b: np.ndarray, tol: float, max_iter: int):
    """Conjugate gradients for apply(x) = b with apply symmetric positive
    definite, from x = 0.  Returns (x, steps, residual norms |r_0|..|r_steps|)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(np.sum(r * r))
    bb = rr
    norms = [math.sqrt(rr)]
    k = 0
    while k < max_iter and rr > tol * tol * bb:
        q = apply(p)
        alpha = rr / float(np.sum(p * q))
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(np.sum(r * r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        norms.append(math.sqrt(rr))
        k += 1
    return x, k, norms


def percentile(x: np.ndarray, pct: float) -> float:
    """pct-th percentile of all values of x: sort, position pct/100 (n - 1),
    linear interpolation between the two neighbouring order statistics."""
    v = np.sort(np.asarray(x, dtype=np.float64).ravel())
    pos = pct / 100.0 * (v.size - 1)
    i = int(math.floor(pos))
    f = pos - i
    if i + 1 >= v.size:
        return float(v[-1])
    return float(v[i] + f * (v[i + 1] - v[i]))


def percentile_clamp(x: np.ndarray, pct: float):
    """Values below the pct-th percentile raised to it; returns (x', q)."""
    q = percentile(x, pct)
    return np.maximum(np.asarray(x, dtype=np.float64), q), q


def noise_sigma(x: np.ndarray) -> float:
    """sqrt of the population variance over all pixels (two passes)."""
    x = np.asarray(x, dtype=np.float64)
    m = float(np.mean(x))
    return math.sqrt(float(np.mean((x - m) ** 2)))


def zeroshot_pnp(u, h, radius, n_it, nu0, tol=1e-3, max_iter=10000, clip_pct=5.0, sigma_px=0.5, radius_d=2,
                 method="auto", which="trace", grad=(1.0, 1.0)):
    """The ZeroShot-PnP deconvolution of the trace image u.  clip_pct None
    disables trimming, sigma_px None makes the denoiser the identity.
    Returns (rho_2, info) with the CG step counts, the noise estimates, the
    nu used by every pass and lambda."""
    u = np.asarray(u, dtype=np.float64)
    taps = trace_taps(u.shape[0], h, radius, which, grad)   # the table of C, built once
    apply_c = lambda x: conv(x, taps, method)
    cu = apply_c(u)                                   # C^T u (C symmetric)
    rho2 = np.zeros_like(u)
    nu = nu0
    lam = None
    info = {"cg_steps": [], "sigma": [], "nu": [], "lam": None}
    for k in range(n_it + 1):
        normal = lambda x, nu=nu: apply_c(apply_c(x)) + nu * x
        rho1, steps, _ = cg(normal, cu + nu * rho2, tol, max_iter)
        if clip_pct is not None:
            rho1, _ = percentile_clamp(rho1, clip_pct)
        sigma = noise_sigma(rho1)
        if k == 0:
            lam = nu0 * sigma * sigma
        rho2 = denoise(rho1, sigma_px, radius_d) if sigma_px is not None else rho1
        info["cg_steps"].append(steps)
        info["sigma"].append(sigma)
        info["nu"].append(nu)
        if sigma > 0.0:
            nu = lam / (sigma * sigma)
    info["lam"] = lam
    return rho2, info
