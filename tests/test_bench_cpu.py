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


def test_cpu_baseline_record_on_a_small_case():
    import bench
    from meshgen import config_case
    case = config_case("c3", n=16, nxy=8)
    rec = bench.cpu_baseline(case, 10, 1, 0.5, sample_iters=3)
    assert rec["kind"] == "oracle" and rec["unit"] == "s" and rec["cores"] == 1
    assert rec["value"] > 0 and rec["oracle_amul_s"] > 0 and rec["oracle_gamg_build_s"] > 0
    assert abs(rec["coe_vs_serial_oracle"] - rec["value"] / 0.5) <= 1e-12 * rec["value"]
    # the sample names the measured size, the iteration count and the sweeps
    assert "measured at 1,024 cells" in rec["sample"]
    assert "3 CG iterations with one 1+1-sweep V-cycle" in rec["sample"]
    assert "times the GPU's 10 iterations" in rec["sample"]


def test_cpu_baseline_names_the_hierarchy():
    import bench
    from meshgen import config_case
    case = config_case("c3", n=16, nxy=8)
    rec = bench.cpu_baseline(case, 10, 1, 0.5, sample_iters=2,
                             hierarchy=bench.HIERARCHIES["aggressive"])
    assert "'passes': 3, 'aggressive_from': 1" in rec["sample"]
    assert rec["value"] > 0
