"""GPU test of the allocation-free pair entry (mpi_batch_pair_noalloc): its
results against the pair entry with caller-owned work memory (bitwise: the
same kernels in the same order) and against the float64 oracle (1e-5), on
two calls in a row, the second with a smaller input, so that the second runs
on the array the first left behind.  A plan whose work memory exceeds the
array is refused on the host (MPI_ERR_WORKSPACE) before anything runs."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2505_22797_amd import mpik
from paper_2505_22797_amd import synth as S
from gpu_helpers import dev, max_rel, rel_l2, rounded

pytestmark = pytest.mark.gpu


def _specs(shapes, seed):
    out = []
    for i, (n, R, t, mode) in enumerate(shapes):
        tr = S.lissajous(t, ax=0.85 - 0.02 * i, ay=0.85)
        out.append(dict(n=n, h=S.h_fwhm2(n) * (0.95 + 0.05 * i), R=R, mode=mode,
                        r=rounded(tr.r, torch.float32), v=rounded(tr.v, torch.float32),
                        c=rounded(S.ellipses_and_line(n, seed + i), torch.float32)))
    return out


def _check(specs):
    batch = mpik.Batch([(sp["n"], sp["h"], sp["R"], dev(sp["r"], torch.float32), dev(sp["v"], torch.float32),
                         sp["mode"]) for sp in specs], tune=False)
    assert batch.work.numel() <= mpik.NOALLOC_SCRATCH_BYTES
    c_all = torch.cat([dev(sp["c"], torch.float32).reshape(-1) for sp in specs])
    s_na = torch.full((batch.s_offsets[-1],), float("nan"), dtype=torch.float32, device="cuda")
    g_na = torch.full((batch.c_offsets[-1],), float("nan"), dtype=torch.float32, device="cuda")
    batch.pair_noalloc(c_all, s_na, g_na)
    s_ref, g_ref = batch.pair(c_all)
    torch.cuda.synchronize()
    assert torch.equal(s_na, s_ref) and torch.equal(g_na, g_ref)
    for b, sp in enumerate(specs):
        M = O.Model(sp["n"], sp["h"], sp["R"], sp["r"], sp["v"])
        s_o = M.forward(sp["c"])
        s_got = batch.s_views(s_na)[b].double().cpu().numpy()
        g_o = M.adjoint(rounded(s_got, torch.float32))
        g_got = batch.c_views(g_na)[b].double().cpu().numpy()
        assert rel_l2(s_got, s_o) <= 1e-5 and max_rel(s_got, s_o) <= 1e-5, b
        assert rel_l2(g_got, g_o) <= 1e-5 and max_rel(g_got, g_o) <= 1e-5, b
    return batch


def test_noalloc_pair_two_calls_then_smaller():
    # first call: three problems (two FFT sizes and the direct path)
    big = _check(_specs([(200, 199, 20000, "fft"), (96, 31, 15000, "direct"), (64, 63, 8000, "fft")], 7100))
    # second call: one smaller problem, on the array the first call left
    small = _check(_specs([(48, 47, 3000, "fft")], 7200))
    assert small.work.numel() < big.work.numel()


def test_noalloc_pair_refuses_a_plan_larger_than_the_array():
    P = S.headline()
    r = dev(S.to_f32(P.traj.r), torch.float32)
    v = dev(S.to_f32(P.traj.v), torch.float32)
    batch = mpik.Batch([(P.n, P.h, P.radius, r, v, "fft")] * 16, tune=False)
    assert batch.work.numel() > mpik.NOALLOC_SCRATCH_BYTES
    c_all = torch.zeros(batch.c_offsets[-1], dtype=torch.float32, device="cuda")
    s_all = torch.zeros(batch.s_offsets[-1], dtype=torch.float32, device="cuda")
    g_all = torch.zeros(batch.c_offsets[-1], dtype=torch.float32, device="cuda")
    with pytest.raises(mpik.MpiError) as err:
        batch.pair_noalloc(c_all, s_all, g_all)
    assert err.value.status == mpik.MPI_ERR_WORKSPACE
