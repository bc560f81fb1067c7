"""Injected resource failures on the GPU (the mpi_debug_fail_alloc hook).

Every resource point of a batch build -- the host allocations of the sizing,
the plan object and the build, the side streams and fork/join events of the
problem ranges -- and of the graph-replayed iteration -- the graph keys and
the captured graphs -- is failed in turn.  Each failing call must return
MPI_ERR_ALLOC (host memory) or MPI_ERR_HIP (stream, event, graph) without
leaving a half-built plan or graph behind, and the first call that gets
through must compute bit for bit what a call that never failed computes.
The failures are forced from the host; no kernel sees anything unusual.
"""
import pytest
import torch

from paper_2505_22797_amd import mpik
from paper_2505_22797_amd import synth as S
from gpu_helpers import dev

pytestmark = pytest.mark.gpu


def _specs(count=16):
    out = []
    for i in range(count):
        tr = S.lissajous(4000 + 100 * i)
        out.append((64, S.h_fwhm2(64), 63, dev(S.to_f32(tr.r), torch.float32), dev(S.to_f32(tr.v), torch.float32),
                    "fft"))
    return out


def _c_all(batch):
    return torch.cat([dev(S.to_f32(S.blobs(n, 50 + b)), torch.float32).reshape(-1) for b, n in enumerate(batch.ns)])


def _until_through(L, attempt, limit=200):
    """Arms the hook at k = 1, 2, ... until `attempt` gets through; returns the
    statuses of the failed attempts and the successful result."""
    codes = []
    try:
        for k in range(1, limit):
            assert L.mpi_debug_fail_alloc(k) == 0
            try:
                out = attempt()
            except mpik.MpiError as e:
                assert e.status in (mpik.MPI_ERR_ALLOC, mpik.MPI_ERR_HIP), (k, e.status)
                codes.append(e.status)
                continue
            return codes, out
        raise AssertionError("the hook never let the call through")
    finally:
        L.mpi_debug_fail_alloc(0)


def test_every_build_failure_point_unwinds(gpu):
    specs = _specs()
    ref = mpik.Batch(specs, tune=False)
    c_all = _c_all(ref)
    s_ref, g_ref = ref.pair(c_all)
    codes, batch = _until_through(ref._L, lambda: mpik.Batch(specs, tune=False))
    print(f"build failure points: {len(codes)} ({codes.count(mpik.MPI_ERR_ALLOC)} host allocations)", flush=True)
    assert mpik.MPI_ERR_ALLOC in codes and mpik.MPI_ERR_HIP in codes
    s, g = batch.pair(c_all)
    torch.cuda.synchronize()
    assert torch.equal(s, s_ref) and torch.equal(g, g_ref)
    batch.close()
    ref.close()


def test_every_graph_failure_point_unwinds(gpu):
    specs = _specs(4)
    ref = mpik.Batch(specs, tune=False)
    batch = mpik.Batch(specs, tune=False)
    c_all = _c_all(ref)
    s = ref.forward(c_all)
    taus = [1e-4] * len(specs)
    x_ref = torch.zeros_like(c_all)
    ref.iterate(s, x_ref, 9, taus, 0.5, 2)            # one block of 8 from a graph, then one single step
    xs = []

    def attempt():
        x = torch.zeros_like(c_all)                   # a new buffer each time: the graphs are re-recorded
        xs.append(x)
        batch.iterate(s, x, 9, taus, 0.5, 2)
        return x

    codes, x = _until_through(batch._L, attempt)
    print(f"graph failure points: {len(codes)}", flush=True)
    assert mpik.MPI_ERR_ALLOC in codes and mpik.MPI_ERR_HIP in codes
    torch.cuda.synchronize()
    assert torch.equal(x, x_ref)
    for failed in xs[:-1]:
        assert not failed.any()                       # a failed call ran no iteration
    x2 = torch.zeros_like(c_all)
    batch.iterate(s, x2, 9, taus, 0.5, 2)
    torch.cuda.synchronize()
    assert torch.equal(x2, x_ref)
    batch.close()
    ref.close()
