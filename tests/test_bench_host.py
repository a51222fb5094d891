"""Host-side checks of bench.py: argument handling and the flop count it reports."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("m", [2, 3, 4, 5, 8, 12, 16])
def test_runtime_T_is_the_walks_swap_cost(m):
    """The flop count bench.py reports, the closed form T(m) of Sec. 5, equals the paper's
    per-swap cost 6 (m - i + 1) of a swap at positions (i, i+1), summed over the swap
    sequence the planner emits for one whole walk."""
    import paper_1901_07643_amd as gs
    seq = gs.upsilon(m)
    assert len(seq) == 2 ** m - m - 1
    assert bench.runtime_T(m) == sum(6 * (m - i + 1) for i in seq)


def test_host_info_fields():
    h = bench.host_info()
    assert set(h) == {"cpu_model", "host_threads", "git_rev", "source_sha16"}
    assert h["host_threads"] >= 1 and len(h["source_sha16"]) == 16
