"""bench.py's contract on the host: more than one GPU is refused before any
GPU is touched, and the algorithmic work behind `roofline.achieved` follows
the per-pair count (28 flop per cell and far node, as the fp32 far term
computes it, 11 per near cell pair,
the group's own 64 self pairs excluded)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_work_count():
    sys.path.insert(0, ROOT)
    import bench

    # group 0: one far node, one near bottom node (its own 8 cells: 512 pairs less the 64 self pairs);
    # group 1: two far nodes
    flops, far, near = bench.algorithmic_flops([1, 2], [1, 0])
    assert far == 64 * 3 and near == 512 - 64
    assert flops == 28 * 192 + 11 * 448
