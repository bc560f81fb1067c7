"""Seeded synthetic inputs: phantoms, field-free-point trajectories and noise.

This module is shared by the GPU path's tests and benchmark and by the CPU
oracle's tests.  It contains none of the operator's arithmetic (no Langevin
function, kernel, convolution, interpolation or transpose): it only draws
concentrations, trajectory samples r_k, velocities v_k = dr/dt and noise, so
that both sides consume identical inputs.

Conventions (the paper fixes none of them for a dimensionless setting):
  * field of view [-1, 1]^2, N x N cell-centred grid, pitch delta = 2/N,
    centres x_i = -1 + (i + 1/2) delta, arrays indexed c[j, i] with j = y;
  * time normalised to one period of the base Lissajous figure, t in [0, 1);
  * sample times t_k = t0 + k (t1 - t0) / T, endpoint excluded;
  * every generator works in float64; callers round to float32 once.

The trajectory shapes follow the paper: the sinusoidal Lissajous scan of its
Experiment 1 (Section "Data", eq. lissajous, frequency dividers 102:96 of
Table 1, i.e. 17:16 cycles per period, 1632 samples per period) and the
drive-plus-excitation scan of Experiment 2 (Section "Experiment 2", the
trajectory equation there).  Velocities are the analytic time derivatives.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Half-maximum radius of the 2-D trace kernel for h = 1: kappa(r*) = kappa(0)/2.
# Choosing h = delta / R_HALF puts the half maximum one pixel from the centre,
# i.e. a point-spread full width at half maximum of two pixels.  The value is
# pinned independently in the oracle tests (mpmath root of the trace kernel).
R_HALF = 2.914188620820050

SAMPLES_PER_PERIOD = 1632          # Table 1, "Sampling points"
LISSAJOUS_CYCLES = (17, 16)        # 2.5 MHz / 102 and 2.5 MHz / 96 over 1632 samples
AMPLITUDE = 0.9


def pitch(n: int) -> float:
    return 2.0 / n


def centres(n: int) -> np.ndarray:
    return -1.0 + (np.arange(n) + 0.5) * pitch(n)


def h_fwhm2(n: int) -> float:
    """Kernel resolution h giving a two-pixel FWHM point-spread at grid n."""
    return pitch(n) / R_HALF


# ----------------------------------------------------------------------------
# trajectories
# ----------------------------------------------------------------------------
@dataclass
class Trajectory:
    t: np.ndarray      # [T]
    r: np.ndarray      # [T, 2] positions (x, y)
    v: np.ndarray      # [T, 2] velocities dr/dt
    kind: str = "lissajous"
    params: dict = field(default_factory=dict)


def sample_times(n_samples: int, t0: float = 0.0, t1: float = 1.0) -> np.ndarray:
    return t0 + np.arange(n_samples, dtype=np.float64) * ((t1 - t0) / n_samples)


def lissajous(n_samples: int, ax: float = AMPLITUDE, ay: float = AMPLITUDE,
              fx: float = LISSAJOUS_CYCLES[0], fy: float = LISSAJOUS_CYCLES[1],
              t0: float = 0.0, t1: float = 1.0,
              exc_amp: float = 0.0, exc_cycles: float = 0.0) -> Trajectory:
    """r(t) = (ax sin 2 pi fx t + exc_amp sin 2 pi exc_cycles t, ay sin 2 pi fy t)."""
    t = sample_times(n_samples, t0, t1)
    w = 2.0 * math.pi
    rx = ax * np.sin(w * fx * t)
    vx = ax * w * fx * np.cos(w * fx * t)
    if exc_amp != 0.0:
        rx = rx + exc_amp * np.sin(w * exc_cycles * t)
        vx = vx + exc_amp * w * exc_cycles * np.cos(w * exc_cycles * t)
    ry = ay * np.sin(w * fy * t)
    vy = ay * w * fy * np.cos(w * fy * t)
    kind = "perturbed" if exc_amp != 0.0 else "lissajous"
    if (t0, t1) != (0.0, 1.0):
        kind += "+window"
    return Trajectory(t, np.stack([rx, ry], 1), np.stack([vx, vy], 1), kind,
                      dict(ax=ax, ay=ay, fx=fx, fy=fy, t0=t0, t1=t1,
                           exc_amp=exc_amp, exc_cycles=exc_cycles))


def experiment2(n_samples: int, ax: float = 0.8, ay: float = 0.85, ae: float = 0.05, fx: float = 50.0,
                fy: float = 1.0, fe: float = 25000.0) -> Trajectory:
    """The non-Lissajous figure of Section "Experiment 2", over one period of
    the slow y drive: r(t) = (ax sin 2 pi fx t + ae sin 2 pi fe t, ay sin 2 pi
    fy t) (the y drive at f_y, the reading of the printed formula), sampled at
    n_samples points; v is the analytic derivative (the experiment itself
    takes forward differences of the positions)."""
    t = sample_times(n_samples)
    w = 2.0 * math.pi
    rx = ax * np.sin(w * fx * t) + ae * np.sin(w * fe * t)
    vx = ax * w * fx * np.cos(w * fx * t) + ae * w * fe * np.cos(w * fe * t)
    ry = ay * np.sin(w * fy * t)
    vy = ay * w * fy * np.cos(w * fy * t)
    return Trajectory(t, np.stack([rx, ry], 1), np.stack([vx, vy], 1), "experiment2",
                      dict(ax=ax, ay=ay, ae=ae, fx=fx, fy=fy, fe=fe))


def trajectory_independence(n_samples: int = 1 << 17) -> Trajectory:
    """Lissajous 17:16 plus an x excitation of amplitude 0.05 at 40x the x
    frequency, observed on the window t in [0, 0.6) (partial data)."""
    return lissajous(n_samples, t0=0.0, t1=0.6, exc_amp=0.05, exc_cycles=40 * 17)


# ----------------------------------------------------------------------------
# phantoms
# ----------------------------------------------------------------------------
def blobs(n: int, seed: int = 0, count: int = 3) -> np.ndarray:
    """Gaussian blobs: centres U[-0.7,0.7]^2, sigma U[1,3] px, amplitude U[0.2,1]."""
    rng = np.random.default_rng(seed)
    d = pitch(n)
    x = centres(n)
    X, Y = np.meshgrid(x, x)           # X[j, i] = x_i, Y[j, i] = y_j
    c = np.zeros((n, n))
    for _ in range(count):
        cx, cy = rng.uniform(-0.7, 0.7, 2)
        sig = rng.uniform(1.0, 3.0) * d
        amp = rng.uniform(0.2, 1.0)
        c += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sig * sig))
    return c


def bars(n: int, gap: float, length: float = 0.5, width: float = 0.06) -> np.ndarray:
    """Two parallel vertical bars `gap` apart (field-of-view units, edge to
    edge), the resolution phantoms of the experiments."""
    x = centres(n)
    X, Y = np.meshgrid(x, x)
    c = np.zeros((n, n))
    for sign in (-1.0, 1.0):
        xc = sign * (gap + width) / 2.0
        c[(np.abs(X - xc) <= width / 2.0) & (np.abs(Y) <= length / 2.0)] = 1.0
    return c


def ellipses_and_line(n: int, seed: int = 0, count: int = 6) -> np.ndarray:
    """Additive ellipses (centres U[-0.6,0.6]^2, semi-axes U[4,16] px, angle
    U[0,pi), value U[0,1]) plus a one-pixel line from (-0.6,-0.5) to (0.5,0.6)
    whose cells (centres within half a pixel of the segment) are set to 1."""
    rng = np.random.default_rng(seed)
    d = pitch(n)
    x = centres(n)
    X, Y = np.meshgrid(x, x)
    c = np.zeros((n, n))
    for _ in range(count):
        cx, cy = rng.uniform(-0.6, 0.6, 2)
        a, b = rng.uniform(4.0, 16.0, 2) * d
        th = rng.uniform(0.0, math.pi)
        val = rng.uniform(0.0, 1.0)
        u = (X - cx) * math.cos(th) + (Y - cy) * math.sin(th)
        w = -(X - cx) * math.sin(th) + (Y - cy) * math.cos(th)
        c += val * ((u / a) ** 2 + (w / b) ** 2 <= 1.0)
    p0 = np.array([-0.6, -0.5])
    p1 = np.array([0.5, 0.6])
    seg = p1 - p0
    lam = np.clip(((X - p0[0]) * seg[0] + (Y - p0[1]) * seg[1]) / (seg @ seg), 0.0, 1.0)
    dist = np.hypot(X - (p0[0] + lam * seg[0]), Y - (p0[1] + lam * seg[1]))
    c[dist <= 0.5 * d] = 1.0
    return c


# ----------------------------------------------------------------------------
# noise
# ----------------------------------------------------------------------------
def add_noise(s: np.ndarray, snr_db: float, seed: int = 1) -> np.ndarray:
    """s + n with n i.i.d. Gaussian over all entries, scaled so that
    10 log10(|s|^2 / |n|^2) = snr_db exactly."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(s.shape)
    scale = np.linalg.norm(s) / (np.linalg.norm(z) * 10.0 ** (snr_db / 20.0))
    return s + scale * z


def unit_directions(shape, count: int, seed: int) -> np.ndarray:
    """Seeded random unit-norm directions (finite-difference probes)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((count,) + tuple(shape))
    return z / np.linalg.norm(z.reshape(count, -1), axis=1).reshape((count,) + (1,) * len(shape))


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    n: int
    h: float
    radius: int
    c: np.ndarray            # [N, N] float64 concentration (ground truth)
    traj: Trajectory
    dtype: str = "f32"
    snr_db: float | None = None
    n_iter: int = 0
    denoise: bool = False
    seed: int = 0

    @property
    def n_samples(self) -> int:
        return self.traj.r.shape[0]


def plain_f64() -> Problem:
    """32x32 grid, three Gaussian blobs, kernel window 15x15, one Lissajous
    period of 4352 samples, noiseless, 50 Landweber iterations, float64."""
    n = 32
    return Problem("plain_f64_32", n, h_fwhm2(n), 7, blobs(n, 0),
                   lissajous(4352), dtype="f64", snr_db=None, n_iter=50, denoise=False)


def plain_f32() -> Problem:
    """128x128 grid, ellipses plus line, window 63x63, 53,856 samples
    (33 periods of 1632), 20 dB noise, 200 denoised gradient iterations."""
    n = 128
    return Problem("plain_f32_128", n, h_fwhm2(n), 31, ellipses_and_line(n, 0),
                   lissajous(33 * SAMPLES_PER_PERIOD), snr_db=20.0, n_iter=200, denoise=True)


def headline(radius: int = 255) -> Problem:
    """256x256 grid, 53,856 Lissajous samples, full-size kernel (R = N-1)."""
    n = 256
    return Problem("headline_256", n, h_fwhm2(n), radius, ellipses_and_line(n, 0),
                   lissajous(33 * SAMPLES_PER_PERIOD), snr_db=20.0, n_iter=200, denoise=True)


def independence() -> Problem:
    """256x256, perturbed partial trajectory with 2^17 samples, full kernel."""
    n = 256
    return Problem("independence_256", n, h_fwhm2(n), 255, ellipses_and_line(n, 0),
                   trajectory_independence(1 << 17), snr_db=20.0, n_iter=200, denoise=True)


def batch_problems(count: int = 64, seed: int = 4, radius: int = 31) -> list[Problem]:
    """Uneven batch: N from {64,96,128,192,256}, T in [10k,120k], kinds
    cycling Lissajous / perturbed / partial, h within +-20% of the 2-px rule."""
    rng = np.random.default_rng(seed)
    sizes = (64, 96, 128, 192, 256)
    out = []
    for b in range(count):
        n = int(sizes[rng.integers(0, len(sizes))])
        t = int(rng.integers(10_000, 120_001))
        kind = b % 3
        hmul = rng.uniform(0.8, 1.2)
        if kind == 0:
            tr = lissajous(t)
        elif kind == 1:
            amp = rng.uniform(0.02, 0.05)
            cyc = 17 * int(rng.integers(20, 61))
            tr = lissajous(t, exc_amp=amp, exc_cycles=cyc)
        else:
            ln = rng.uniform(0.4, 0.8)
            t0 = rng.uniform(0.0, 1.0 - ln)
            tr = lissajous(t, t0=t0, t1=t0 + ln)
        out.append(Problem(f"batch_{b}", n, h_fwhm2(n) * hmul, radius,
                           ellipses_and_line(n, 1000 + b), tr, snr_db=20.0,
                           n_iter=50, denoise=True, seed=1000 + b))
    return out


def gradient_problems(count: int = 8) -> list[Problem]:
    """Problems at 256^2 with 53,856 samples and a 63x63 window."""
    n = 256
    return [Problem(f"grad_{b}", n, h_fwhm2(n), 31, ellipses_and_line(n, 2000 + b),
                    lissajous(33 * SAMPLES_PER_PERIOD), snr_db=20.0, n_iter=20,
                    denoise=True, seed=2000 + b) for b in range(count)]


def to_f32(a: np.ndarray) -> np.ndarray:
    """Round once to float32 and return the rounded values as float64."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)
