"""GPU tests of the plan build: the samples' order in the plan is the stable
sort by base cell of the time indices, with the base cells the oracle's
bilinear rule gives.  Sizes cover one, two and three radix passes, tiles with
a ragged tail and cells holding thousands of samples."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2505_22797_amd import mpik
from paper_2505_22797_amd import synth as S
from gpu_helpers import dev, rounded

pytestmark = pytest.mark.gpu


def _trajectories():
    yield 2, S.lissajous(100, ax=0.45, ay=0.45)                       # a single cell
    yield 16, S.lissajous(3001, ax=0.85, ay=0.8)
    yield 16, S.lissajous(60000, ax=0.85, ay=0.8, fx=3, fy=2)        # about 270 samples per cell
    yield 256, S.lissajous(53856)                                     # 27 tiles, the last one ragged
    yield 300, S.lissajous(20000, ax=0.8, ay=0.85, exc_amp=0.05, exc_cycles=17 * 40)   # 3 passes
    tr = S.lissajous(5000, ax=0.5, ay=0.5)
    yield 64, S.Trajectory(tr.t, np.full_like(tr.r, 0.123), tr.v, "still", {})            # one cell, 3 tiles


@pytest.mark.parametrize("case", range(6))
def test_sample_order_is_stable_sort_by_cell(case):
    n, tr = list(_trajectories())[case]
    r = rounded(tr.r, torch.float32)
    v = rounded(tr.v, torch.float32)
    plan = mpik.Plan(n, S.h_fwhm2(n), 3, dev(r, torch.float32), dev(v, torch.float32), conv_mode="direct")
    order, cell = plan.sample_order()
    torch.cuda.synchronize()
    ix, jy, _, _ = O.bilinear(r, n)
    key = jy * (n - 1) + ix
    ref = np.lexsort((np.arange(r.shape[0]), key))
    assert np.array_equal(order.cpu().numpy(), ref)
    assert np.array_equal(cell.cpu().numpy(), (ix | (jy << 16))[ref])
