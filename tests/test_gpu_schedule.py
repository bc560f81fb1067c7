"""The launch schedule of a batch (mpi_batch_schedule): problem ranges per
FFT-size group on their own side streams.  Every range count gives the pair
bit for bit, and the cached iteration graphs follow a change of schedule.
The timed choice of the count is switched off (its test is skipped)."""
import pytest
import torch

from paper_2505_22797_amd import mpik
from paper_2505_22797_amd import synth as S
from gpu_helpers import dev

pytestmark = pytest.mark.gpu


def _batch(sizes):
    specs = []
    for i, n in enumerate(sizes):
        tr = S.lissajous(3000 + 211 * i)
        specs.append((n, S.h_fwhm2(n), n - 1, dev(S.to_f32(tr.r), torch.float32), dev(S.to_f32(tr.v), torch.float32),
                      "fft"))
    batch = mpik.Batch(specs, tune=False)
    c_all = torch.cat([dev(S.to_f32(S.blobs(n, 80 + i)), torch.float32).reshape(-1) for i, n in enumerate(sizes)])
    return batch, c_all


@pytest.mark.parametrize("sizes,default,top", [([64] * 20, 4, 8), ([64] * 10 + [128] * 10, 2, 4)])
def test_every_range_count_gives_the_same_pair(gpu, sizes, default, top):
    batch, c_all = _batch(sizes)
    assert batch.schedule() == default
    s_ref, g_ref = batch.pair(c_all)
    torch.cuda.synchronize()
    s_ref, g_ref = s_ref.clone(), g_ref.clone()
    r = 1
    while r <= top:
        assert batch.schedule(r) == r
        s, g = batch.pair(c_all)
        torch.cuda.synchronize()
        assert torch.equal(s, s_ref) and torch.equal(g, g_ref), r
        r *= 2
    with pytest.raises(mpik.MpiError):
        batch.schedule(top + 1)
    batch.close()


@pytest.mark.skip(reason="choosing the range count by timing is switched off in the library: its graph-captured "
                         "timing runs once ended in a host-side fault whose cause is not established")
def test_timed_range_choice_keeps_the_results(gpu):
    batch, c_all = _batch([64] * 10 + [128] * 10)
    s_ref, g_ref = batch.pair(c_all)
    torch.cuda.synchronize()
    s_ref, g_ref = s_ref.clone(), g_ref.clone()
    chosen = batch.schedule(0, c_all)
    assert chosen in (1, 2, 4) and batch.schedule() == chosen
    s, g = batch.pair(c_all)
    torch.cuda.synchronize()
    assert torch.equal(s, s_ref) and torch.equal(g, g_ref)
    batch.close()


def test_iteration_graphs_follow_the_schedule(gpu):
    batch, c_all = _batch([64] * 16)
    s = batch.forward(c_all)
    taus = [1e-4] * 16
    x_ref = torch.zeros_like(c_all)
    batch.iterate(s, x_ref, 9, taus, 0.5, 2)        # records the graphs with four ranges
    for r in (1, 8, 2):
        batch.schedule(r)
        x = torch.zeros_like(c_all)
        batch.iterate(s, x, 9, taus, 0.5, 2)
        x2 = torch.zeros_like(c_all)
        batch.iterate(s, x2, 9, taus, 0.5, 2)         # replays the graphs recorded for r
        torch.cuda.synchronize()
        assert torch.equal(x, x_ref) and torch.equal(x2, x_ref), r
    batch.close()
