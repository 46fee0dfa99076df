"""Host-side parts of bench.py, on the CPU: the one-GPU guard and the cluster sample the
oracle baseline runs on for the largest workload."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_baseline_sample_holds_whole_clusters_and_the_largest():
    rng = np.random.default_rng(1)
    sizes = np.concatenate([rng.integers(11, 3000, 5000), rng.integers(3001, 50000, 40),
                            [999_269, 400_000, 250_000, 120_000]])
    memb = np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)
    memb = np.concatenate([memb, np.full(1000, -1, np.int32)])   # unassigned vertices
    pick = bench.sample_clusters(memb)
    assert len(pick) == len(np.unique(pick)) == 400 + 6 + 3
    top3 = np.argsort(-sizes)[:3]
    assert set(top3.tolist()) <= set(pick.tolist())
    assert sizes[pick].max() == 999_269
    # the same sample every time (seeded)
    assert np.array_equal(pick, bench.sample_clusters(memb))
