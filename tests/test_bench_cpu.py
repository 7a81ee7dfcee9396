"""Host-side checks of bench.py: the one-GPU guard and the oracle baseline
record (run on a small slab of the graded workload; no GPU is touched)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "--gpus must be 1" in json.loads(p.stdout.strip().splitlines()[-1])["error"]


def test_cpu_baseline_record_on_a_small_slab():
    import bench
    rec = bench.cpu_baseline(10, n=16, nxy=8, sample_iters=3)
    assert rec["kind"] == "oracle" and rec["unit"] == "s" and rec["cores"] == 1
    assert rec["value"] > 0
    # the sample names its size, its iteration count and the scaling applied
    assert "8x8x16" in rec["sample"] and "3 V-cycle-preconditioned CG iterations" in rec["sample"]
    assert "x10 by the GPU's iteration count" in rec["sample"]
