"""Host-side checks of the benchmark's contract (no GPU): one GPU only, and
the timed step count is exact."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused_with_a_message(n):
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr and out.stdout == ""


@pytest.mark.parametrize("steps", [1, 7, 12, 60, 200, 1000])
def test_graph_groups_divide_the_step_count(steps):
    g = bench.group_for(steps)
    assert steps % g == 0 and g in (1, 2, 4, 5, 8, 10)



@pytest.mark.parametrize("n,t", [(256, 53856), (128, 53856), (32, 4352)])
def test_stage_shares_sum_to_the_pair_bytes(n, t):
    """The per-stage shares of the roofline add up to the algorithmic bytes
    of one pair, 56 N^2 + 48 T in float32."""
    total = sum(bench.alg_stage_bytes(k, n, t) for k in bench.STAGE_NAMES)
    assert total == 56 * n * n + 48 * t
