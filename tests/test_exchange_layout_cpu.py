"""Host check of the register FFT's float32 exchange layout (the slot map in
csrc/common.hpp): a bijection of the 512 elements, and for each of the three
access shapes of the 8 x 8 exchange every group of 16 lanes touches 16
distinct bank pairs (8-byte elements on 32 four-byte banks) and every group of
32 lanes 32 distinct pairs (64 banks).  Also checks the per-lane-part XOR
per-register-constant split the kernel relies on."""
import os
import re

import pytest

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2505_22797_amd", "csrc", "common.hpp")


def _images():
    text = open(SRC).read()
    m = re.search(r"kImage\[9\]\s*=\s*\{([^}]*)\}", text)
    assert m, "float32 exchange images not found"
    return [int(v) for v in m.group(1).split(",")]


def _slot(img, i):
    s = 0
    for b in range(9):
        if (i >> b) & 1:
            s ^= img[b]
    return s


def _shapes():
    """Element index per lane for every register k of the three accesses."""
    out = []
    for k in range(8):
        out.append([64 * k + 8 * (l & 7) + (l >> 3) for l in range(64)])      # lane a + 8b writes (k, a, b)
        out.append([64 * (l & 7) + 8 * (l >> 3) + k for l in range(64)])      # lane lo + 8hi reads (lo, hi, k)
        out.append([64 * (l & 7) + 8 * k + (l >> 3) for l in range(64)])      # lane lo + 8hi writes (lo, k, hi)
    return out


def test_bijection():
    img = _images()
    assert sorted(_slot(img, i) for i in range(512)) == list(range(512))


@pytest.mark.parametrize("group,pairs", [(16, 16), (32, 32)])
def test_conflict_free(group, pairs):
    img = _images()
    for idx in _shapes():
        for g0 in range(0, 64, group):
            banks = [_slot(img, i) % pairs for i in idx[g0:g0 + group]]
            assert len(set(banks)) == group


def test_padding_it_replaces_conflicts():
    """The plain one-in-nine padding is not conflict-free for 8-byte elements
    (so the test above can fail)."""
    worst = 0
    for idx in _shapes():
        for g0 in range(0, 64, 16):
            banks = [(i + (i >> 3)) % 16 for i in idx[g0:g0 + 16]]
            worst = max(worst, 16 - len(set(banks)) + 1)
    assert worst > 1


def test_lane_part_xor_register_constant():
    img = _images()
    s = lambda i: _slot(img, i)
    for lane in range(64):
        lo, hi = lane & 7, lane >> 3
        for k in range(8):
            assert s(64 * k + 8 * lo + hi) == s(8 * lo + hi) ^ s(64 * k)
            assert s(64 * lo + 8 * hi + k) == s(64 * lo + 8 * hi) ^ s(k)
            assert s(64 * lo + 8 * k + hi) == s(64 * lo + hi) ^ s(8 * k)
