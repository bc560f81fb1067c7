"""GPU parity at the library's size limits, against the float64 oracle: the
largest grid (1024^2, direct path) with the largest sample count (2^26 - 1),
and the largest FFT sizes (1024 in float32 on the largest FFT grid, 512^2,
and 512 in float64).  At 2^26 samples the
forward signal is compared on sampled outputs, which the oracle computes one
by one (each sample's value depends on that sample alone), and the transpose
with a signal that is nonzero on those samples only, whose transpose the
oracle computes from them alone."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2505_22797_amd import mpik
from paper_2505_22797_amd import synth as S
from gpu_helpers import max_rel, dev, rel_l2, rounded

pytestmark = pytest.mark.gpu


def test_largest_grid_and_sample_count():
    n, R, t = 1024, 7, (1 << 26) - 1
    tr = S.lissajous(t, ax=0.97, ay=0.96)
    r, v = rounded(tr.r, torch.float32), rounded(tr.v, torch.float32)
    del tr
    h = S.h_fwhm2(n)
    c = rounded(S.blobs(n, 11), torch.float32)
    plan = mpik.Plan(n, h, R, dev(r, torch.float32), dev(v, torch.float32), conv_mode="direct")
    s = plan.forward(dev(c, torch.float32))
    rng = np.random.default_rng(3)
    pick = np.sort(rng.choice(t, 4096, replace=False))
    got = s[torch.tensor(pick, device="cuda")].double().cpu().numpy()
    sub = O.Model(n, h, R, r[pick], v[pick])
    assert rel_l2(got, sub.forward(c)) <= 1e-5
    y = rounded(rng.standard_normal((pick.size, 2)), torch.float32)
    y_all = torch.zeros((t, 2), dtype=torch.float32, device="cuda")
    y_all[torch.tensor(pick, device="cuda")] = dev(y, torch.float32)
    g = plan.adjoint(y_all).double().cpu().numpy()
    assert rel_l2(g, sub.adjoint(y)) <= 1e-5


@pytest.mark.parametrize("dtype,n,R", [(torch.float32, 512, 511), (torch.float64, 400, 112)])
def test_largest_fft_size(dtype, n, R):
    """The largest FFT each dtype supports: M = 1024 in float32 (the largest
    FFT grid, 512^2, with the full kernel) and M = 512 in float64; forward
    and transpose against the oracle element by element."""
    t = 200_000
    tr = S.lissajous(t, ax=0.9, ay=0.88)
    r, v = rounded(tr.r, dtype), rounded(tr.v, dtype)
    h = S.h_fwhm2(n)
    c = rounded(S.ellipses_and_line(n, 5), dtype)
    plan = mpik.Plan(n, h, R, dev(r, dtype), dev(v, dtype), conv_mode="fft")
    assert plan.fft_size == (1024 if dtype == torch.float32 else 512)
    M = O.Model(n, h, R, r, v)
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    s = plan.forward(dev(c, dtype)).double().cpu().numpy()
    s_ref = M.forward(c)
    assert rel_l2(s, s_ref) <= tol and max_rel(s, s_ref) <= tol
    y = rounded(np.random.default_rng(4).standard_normal((t, 2)), dtype)
    g = plan.adjoint(dev(y, dtype)).double().cpu().numpy()
    g_ref = M.adjoint(y)
    assert rel_l2(g, g_ref) <= tol and max_rel(g, g_ref) <= tol
