"""Host checks of bench.py's contract (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus_requested"] == 2


def test_kernel_costs_of_the_headline_workload():
    sys.path.insert(0, ROOT)
    import bench
    n, p = 400, 5000
    c = bench.kernel_costs(n, p, "mixed")
    nbytes, flops, dt = c["syrk_bf16x3"]
    assert dt == "bf16" and flops == 3.0 * n * p * (p + 1)
    assert nbytes == 4.0 * p * p + 4.0 * 448 * p  # S written once, the bf16 split (448 padded samples) read once
    assert c["kkt_rows"][0] == 4.0 * p * p and c["fill_B"][0] == 8.0 * p * p
    c64 = bench.kernel_costs(n, p, "fp64")
    assert c64["syrk_f64"][1] == float(n) * p * (p + 1) and c64["kkt_rows"][0] == 8.0 * p * p
