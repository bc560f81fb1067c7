"""Seeded random problem shapes through one batch, against the float64 oracle.

Each draw picks a grid side N in [2, 96], a window R in [0, N - 1] (a third
of the draws take the full kernel R = N - 1), a sample count T in [1, 4000]
(T = 1 included), a convolution path (auto, direct up to R = 40, FFT), the
interpolator (bilinear, cosine) and the receive channels (both, x alone).
Sample positions are uniform over the hull of the cell centres, [-(1 - 1/N),
1 - 1/N]^2, with its four corners and edge midpoints always among them: on
the hull exactly when N is a power of two (samples whose weight of the upper
neighbour is exactly 0 or 1), a hair inside otherwise; velocities are
standard normal.  The whole draw runs as one batch (so it also mixes FFT
sizes, paths and interpolators in every launch); s = A c and A^T y of every
problem are compared with the oracle, by relative L2 error and element by
element (max |got - ref| / max |ref|).  Operator: eq. (coreoperator) sampled
and contracted per eq. (core:formula).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2505_22797_amd import mpik
from gpu_helpers import dev, max_rel, rel_l2, rounded

pytestmark = pytest.mark.gpu

TOL = {torch.float32: (1e-5, 1e-5), torch.float64: (1e-13, 1e-13)}   # (rel-L2, element-wise); measured 8e-7, 3e-15


def _draw(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(2, 97))
        R = n - 1 if rng.random() < 1 / 3 else int(rng.integers(0, n))
        t = 1 if i == 0 else int(rng.integers(1, 4001))
        a = 1.0 - 1.0 / n
        # the hull's corners and edge midpoints: exactly on it when N is a power of two (the cell
        # centres are exact binary fractions), else a hair inside, so that rounding never leaves it
        e = a if n & (n - 1) == 0 else a * (1.0 - 2.0 ** -20)
        fixed = np.array([[-e, -e], [e, -e], [-e, e], [e, e], [0.0, -e], [0.0, e], [-e, 0.0], [e, 0.0]])
        r = rng.uniform(-a, a, (t, 2)) * (1.0 - 2.0 ** -20)
        r[: min(t, len(fixed))] = fixed[: min(t, len(fixed))]
        v = rng.standard_normal((t, 2))
        # the direct path keeps its input tile in LDS: windows up to 40 here
        mode = ("auto", "direct", "fft")[int(rng.integers(0, 3))]
        if mode == "direct" and R > 40:
            mode = "fft"
        interp = ("bilinear", "cosine")[int(rng.integers(0, 2))]
        h = (2.0 / n) * rng.uniform(0.6, 2.5)
        out.append(dict(n=n, R=R, t=t, r=r, v=v, mode=mode, interp=interp, h=h,
                        c=rng.standard_normal((n, n)), y=rng.standard_normal((t, 2))))
    return out


@pytest.mark.parametrize("channels", ["xy", "x"])
@pytest.mark.parametrize("dtype,seed", [(torch.float32, 101), (torch.float64, 202)])
def test_random_shapes_match_oracle(gpu, dtype, seed, channels):
    draws = _draw(seed + (7 if channels == "x" else 0), 24)
    for d in draws:
        d["r"], d["v"] = rounded(d["r"], dtype), rounded(d["v"], dtype)
        d["c"], d["y"] = rounded(d["c"], dtype), rounded(d["y"], dtype)
    batch = mpik.Batch([(d["n"], d["h"], d["R"], dev(d["r"], dtype), dev(d["v"], dtype), d["mode"], d["interp"])
                        for d in draws], dtype=dtype, tune=False, channels=channels)
    c_all = torch.cat([dev(d["c"], dtype).reshape(-1) for d in draws])
    y_all = torch.cat([dev(d["y"], dtype).reshape(-1) for d in draws])
    s_all = batch.forward(c_all)
    g_all = batch.adjoint(y_all)
    torch.cuda.synchronize()
    s_v = [x.double().cpu().numpy() for x in batch.s_views(s_all)]
    g_v = [x.double().cpu().numpy() for x in batch.c_views(g_all)]
    l2, el = TOL[dtype]
    worst = [0.0, 0.0]
    for b, d in enumerate(draws):
        M = O.Model(d["n"], d["h"], d["R"], d["r"], d["v"], interp=d["interp"], channels=channels)
        s_ref = M.forward(d["c"])
        g_ref = M.adjoint(d["y"])
        case = (b, d["n"], d["R"], d["t"], d["mode"], d["interp"], batch.info[b]["conv_mode"])
        if np.any(s_ref):
            e = (rel_l2(s_v[b], s_ref), max_rel(s_v[b], s_ref))
            worst[0] = max(worst[0], e[1])
            assert e[0] <= l2 and e[1] <= el, ("forward", case, e)
        else:
            assert not np.any(s_v[b]), ("forward", case)
        if np.any(g_ref):
            e = (rel_l2(g_v[b], g_ref), max_rel(g_v[b], g_ref))
            worst[1] = max(worst[1], e[1])
            assert e[0] <= l2 and e[1] <= el, ("transpose", case, e)
        else:
            assert not np.any(g_v[b]), ("transpose", case)
    print(f"random shapes {dtype} {channels}: paths "
          f"{sorted(set(i['conv_mode'] for i in batch.info))}, worst element-wise forward {worst[0]:.1e}, "
          f"transpose {worst[1]:.1e}", flush=True)
    batch.close()


@pytest.mark.parametrize("dtype,seed", [(torch.float32, 303), (torch.float64, 404)])
def test_random_shapes_vjp_and_iteration(gpu, dtype, seed):
    """The same kind of draw (both receive channels) through the
    composite VJP of s = A c (A^T gs, <(dA/dh) c, gs>, the trajectory
    gradients) and six denoised iterations with tau = 0.9 / lambda_max(A^T A)
    (the oracle's power estimate), against the oracle."""
    draws = _draw(seed, 16)
    for d in draws:
        d["r"], d["v"] = rounded(d["r"], dtype), rounded(d["v"], dtype)
        d["c"], d["y"] = rounded(d["c"], dtype), rounded(d["y"], dtype)
    batch = mpik.Batch([(d["n"], d["h"], d["R"], dev(d["r"], dtype), dev(d["v"], dtype), d["mode"], d["interp"])
                        for d in draws], dtype=dtype, tune=False, deriv=True)
    c_all = torch.cat([dev(d["c"], dtype).reshape(-1) for d in draws])
    y_all = torch.cat([dev(d["y"], dtype).reshape(-1) for d in draws])
    gc, g_h, g_r, g_v = batch.vjp_forward(c_all, y_all)
    models = [O.Model(d["n"], d["h"], d["R"], d["r"], d["v"], interp=d["interp"]) for d in draws]
    taus = [0.9 / max(O.power_lambda_max(M, iters=20), 1e-30) for M in models]
    x_all = torch.zeros_like(c_all)
    batch.iterate(y_all, x_all, 6, taus, 0.5, 2)
    torch.cuda.synchronize()
    gc_v = [x.double().cpu().numpy() for x in batch.c_views(gc)]
    gr_v = [x.double().cpu().numpy() for x in batch.s_views(g_r)]
    gv_v = [x.double().cpu().numpy() for x in batch.s_views(g_v)]
    x_v = [x.double().cpu().numpy() for x in batch.c_views(x_all)]
    gh = g_h.cpu().numpy()
    l2 = TOL[dtype][0]
    it_tol = 1e-4 if dtype == torch.float32 else 1e-11
    for b, d in enumerate(draws):
        M = models[b]
        case = (b, d["n"], d["R"], d["t"], d["mode"], d["interp"])
        ref_gc = M.adjoint(d["y"])
        r_ref, v_ref = M.traj_vjp(d["c"], d["y"])
        dh = M.forward_dh(d["c"]) * d["y"]
        for got, ref, what in ((gc_v[b], ref_gc, "A^T gs"), (gr_v[b], r_ref, "g_r"), (gv_v[b], v_ref, "g_v")):
            if np.any(ref):
                assert rel_l2(got, ref) <= 10 * l2, (what, case, rel_l2(got, ref))
        assert abs(gh[b] - dh.sum()) <= 10 * l2 * max(np.abs(dh).sum(), 1e-300), ("g_h", case, gh[b], dh.sum())
        ref_x = O.iterate(M, d["y"], np.zeros((d["n"], d["n"])), taus[b], 6, sigma_px=0.5, radius=2)
        if np.any(ref_x):
            assert rel_l2(x_v[b], ref_x) <= it_tol, ("iterate", case, rel_l2(x_v[b], ref_x))
    batch.close()
