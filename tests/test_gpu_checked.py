"""The bounds-checked debug build (libmpik_check.so, compiled with
-DMPIK_CHECK) on the GPU.

* On valid plans it reports nothing and computes what the release build
  computes: the headline pair call over 16 problems (problem ranges on side
  streams), and a mixed batch -- both convolution paths, both interpolators,
  float32 -- through the pair, the denoised iteration (graph replay), the
  derivative entries and the Core Stage.
* On a plan whose sample tables were corrupted from the host -- a base cell
  one past the grid, a time index one past the end, a row's sample range
  past the last sample -- each check sets its bit in the problem's check
  word, the access it guards is skipped and every kernel still ends
  normally.  The corrupted values only ever reach the checked kernels.

The whole GPU suite can also run on this build (MPIK_LIBRARY=libmpik_check.so);
conftest then asserts that every plan closes with a zero check word.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2505_22797_amd import mpik
from paper_2505_22797_amd import synth as S
from gpu_helpers import dev, max_rel

pytestmark = pytest.mark.gpu


class ProbDesc(ctypes.Structure):
    """Leading fields of a problem descriptor as the plan memory holds it
    (one per problem at the start of the plan)."""
    _fields_ = [("n", ctypes.c_int32), ("nb", ctypes.c_int32), ("radius", ctypes.c_int32), ("m", ctypes.c_int32),
                ("log2m", ctypes.c_int32), ("mode", ctypes.c_int32), ("taps_w", ctypes.c_int32),
                ("slices", ctypes.c_int32), ("interp", ctypes.c_int32), ("chan", ctypes.c_int32),
                ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("t", ctypes.c_int64), ("h", ctypes.c_double),
                ("o_c", ctypes.c_int64), ("o_s", ctypes.c_int64), ("o_taps", ctypes.c_int64),
                ("o_spec", ctypes.c_int64), ("o_taps_dh", ctypes.c_int64), ("o_spec_dh", ctypes.c_int64),
                ("o_tw", ctypes.c_int64), ("o_samp", ctypes.c_int64), ("o_dw", ctypes.c_int64),
                ("o_sidx", ctypes.c_int64), ("o_binstart", ctypes.c_int64), ("o_err", ctypes.c_int64)]


PROB_BYTES = 232      # sizeof of the whole descriptor


@pytest.fixture(scope="module")
def checked():
    import os
    if not os.path.exists(mpik.CHECK_LIBRARY):
        pytest.fail("libmpik_check.so is missing: build it with `python -m paper_2505_22797_amd.build`")
    with mpik.use_library(mpik.CHECK_LIBRARY) as L:
        assert L.mpi_checks_enabled() == 1
    return mpik.CHECK_LIBRARY


def _both(checked, make):
    """The same object built by the release and the checked library."""
    rel = make()
    with mpik.use_library(checked):
        chk = make()
    return rel, chk


def _same(a, b, tol):
    torch.cuda.synchronize()
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    assert np.all(np.isfinite(b))
    if np.array_equal(a, b):
        return 0.0
    e = max_rel(b, a)
    assert e <= tol, e
    return e


def test_checked_headline_pair_matches_release(checked):
    P = S.headline()
    r, v = dev(S.to_f32(P.traj.r), torch.float32), dev(S.to_f32(P.traj.v), torch.float32)
    B = 16
    rel, chk = _both(checked, lambda: mpik.Batch([(P.n, P.h, P.radius, r, v, "fft")] * B, tune=False))
    c_all = torch.cat([dev(S.to_f32(S.ellipses_and_line(P.n, 7000 + b)), torch.float32).reshape(-1)
                       for b in range(B)])
    s1, g1 = rel.pair(c_all)
    s2, g2 = chk.pair(c_all)
    print(f"checked headline pair: s {_same(s1, s2, 1e-6):.1e} g {_same(g1, g2, 1e-6):.1e}", flush=True)
    assert chk.check_word() == 0
    rel.close()
    chk.close()


def _mixed_specs():
    specs = []
    for i, (n, R, t, mode, interp) in enumerate([(64, 5, 9000, "direct", "bilinear"), (96, 31, 20000, "fft", "cosine"),
                                                 (128, 127, 30000, "fft", "bilinear"),
                                                 (48, 7, 6000, "direct", "cosine")]):
        tr = S.lissajous(t)
        specs.append((n, S.h_fwhm2(n) * (1.0 + 0.05 * i), R, dev(S.to_f32(tr.r), torch.float32),
                      dev(S.to_f32(tr.v), torch.float32), mode, interp))
    return specs


def test_checked_mixed_batch_matches_release(checked):
    specs = _mixed_specs()
    rel, chk = _both(checked, lambda: mpik.Batch(specs, tune=False, deriv=True))
    c_all = torch.cat([dev(S.to_f32(S.blobs(sp[0], 30 + i)), torch.float32).reshape(-1)
                       for i, sp in enumerate(specs)])
    worst = 0.0
    s1, g1 = rel.pair(c_all)
    s2, g2 = chk.pair(c_all)
    worst = max(worst, _same(s1, s2, 1e-6), _same(g1, g2, 1e-6))
    taus = [1e-4] * len(specs)
    x1 = torch.zeros_like(c_all)
    x2 = torch.zeros_like(c_all)
    rel.iterate(s1, x1, 12, taus, 0.5, 2)
    chk.iterate(s1, x2, 12, taus, 0.5, 2)
    worst = max(worst, _same(x1, x2, 1e-5))
    worst = max(worst, _same(rel.forward_dh(c_all), chk.forward_dh(c_all), 1e-6))
    gr1, gv1 = rel.traj_vjp(c_all, s1)
    gr2, gv2 = chk.traj_vjp(c_all, s1)
    worst = max(worst, _same(gr1, gr2, 1e-5), _same(gv1, gv2, 1e-5))
    f1, k1 = rel.core_stage(s1, gamma=1e-3, tol=0.0, max_iter=8)
    f2, k2 = chk.core_stage(s1, gamma=1e-3, tol=0.0, max_iter=8)
    worst = max(worst, _same(f1, f2, 1e-5))
    print(f"checked mixed batch: worst element-wise difference {worst:.1e}", flush=True)
    assert chk.check_word() == 0
    rel.close()
    chk.close()


def _desc(batch, b):
    raw = batch.plan_mem[b * PROB_BYTES:b * PROB_BYTES + ctypes.sizeof(ProbDesc)].cpu().numpy().tobytes()
    d = ProbDesc.from_buffer_copy(raw)
    assert d.n == batch.ns[b] and d.t == batch.ts[b] and d.nb == d.n - 1
    assert d.o_c == batch.c_offsets[b] and d.o_s == batch.s_offsets[b]
    return d


def _poke_i32(batch, byte_off, value):
    batch.plan_mem[byte_off:byte_off + 4].view(torch.int32).fill_(int(value))
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", ["fft", "direct"])
@pytest.mark.parametrize("what,bit", [("cell", 1), ("time", 2), ("range", 4)])
def test_checked_build_flags_corrupt_tables(checked, mode, what, bit):
    n, t = 64, 8000
    tr = S.lissajous(t)
    r, v = dev(S.to_f32(tr.r), torch.float32), dev(S.to_f32(tr.v), torch.float32)
    with mpik.use_library(checked):
        batch = mpik.Batch([(n, S.h_fwhm2(n), 7 if mode == "direct" else 31, r, v, mode)], tune=False)
    assert batch.info[0]["conv_mode"] == mode
    d = _desc(batch, 0)
    order, cell = batch.sample_order(0)
    torch.cuda.synchronize()
    i = t // 2
    sidx = batch.plan_mem[d.o_sidx:d.o_sidx + 8 * t].view(torch.int32).reshape(t, 2)
    assert torch.equal(sidx[:, 0], cell) and torch.equal(sidx[:, 1], order)   # the descriptor read right
    if what == "cell":
        packed = int(cell[i])
        _poke_i32(batch, d.o_sidx + 8 * i, (packed & ~0xffff) | d.nb)          # i0 one past the last base cell
    elif what == "time":
        _poke_i32(batch, d.o_sidx + 8 * i + 4, t)                               # one past the last sample
    else:
        _poke_i32(batch, d.o_binstart + 4 * d.nb * d.nb, t + 1)                 # last row's range past T
    c = dev(S.to_f32(S.blobs(n, 3)), torch.float32).reshape(-1)
    y = torch.zeros(2 * t, dtype=torch.float32, device="cuda")
    s = batch.forward(c)
    batch.adjoint(s)
    x = torch.zeros_like(c)
    batch.iterate(y, x, 2, [1e-4], 0.0, 0)        # time-ordered signal read through the sample table
    torch.cuda.synchronize()                       # every kernel ended normally
    word = batch.check_word()
    assert word & bit, (what, mode, word)
    batch.close()
    assert mpik.CHECK_FAILURES and mpik.CHECK_FAILURES[-1][1] & bit
    mpik.CHECK_FAILURES.clear()
