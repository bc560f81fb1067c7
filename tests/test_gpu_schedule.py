"""The launch schedule of a batch (mpi_batch_schedule): problem ranges per
FFT-size group on their own side streams.  Every range count gives the pair
bit for bit, and a plan that has recorded graphs keeps its schedule.  The
timed choice of the count is switched off, and so is a change of count after
a graph capture (their tests are skipped, with the reasons)."""
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


@pytest.mark.skip(reason="a graph-replayed iteration recorded after a change of schedule (side streams destroyed "
                         "and re-created after an earlier capture) ended the process with a host segmentation "
                         "fault; no cause is established, so the library refuses such a change once a plan has "
                         "recorded graphs (test_schedule_is_kept_once_graphs_are_recorded)")
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


def test_schedule_is_kept_once_graphs_are_recorded(gpu):
    """A plan that has recorded graphs keeps its range count: a different
    count is refused with MPI_ERR_UNSUPPORTED (nothing is re-created), the
    same count is accepted, and the cached graphs keep replaying the same
    results."""
    batch, c_all = _batch([64] * 16)
    assert batch.schedule() == 4                      # the build's count for 16 problems of one size
    s = batch.forward(c_all)
    taus = [1e-4] * 16
    x_ref = torch.zeros_like(c_all)
    batch.iterate(s, x_ref, 9, taus, 0.5, 2, use_graph=False)
    x = torch.zeros_like(c_all)
    batch.iterate(s, x, 9, taus, 0.5, 2)             # records the graphs
    for r in (1, 2, 8):
        with pytest.raises(mpik.MpiError) as ei:
            batch.schedule(r)
        assert ei.value.status == mpik.MPI_ERR_UNSUPPORTED
    assert batch.schedule(4) == 4 and batch.schedule() == 4
    x2 = torch.zeros_like(c_all)
    batch.iterate(s, x2, 9, taus, 0.5, 2)            # new buffer: recorded again, same streams
    torch.cuda.synchronize()
    assert torch.equal(x, x_ref) and torch.equal(x2, x_ref)
    batch.close()
