"""bench.py on the CPU: a run on more than one GPU is refused with a message
(one process drives one GPU), and every workload's solve parameters ask for
the metric's residual."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "--gpus must be 1" in msg["error"]


def test_every_workload_solves_to_the_metric_residual():
    sys.path.insert(0, ROOT)
    import bench

    for p in (bench.SOLVE, bench.RGG_SOLVE, bench.SERVE_SOLVE, bench.BATCH_SOLVE,
              bench.SQUARE_SOLVE, bench.PARTITION_SOLVE, bench.GS_SOLVE):
        assert p["tol_res"] == 1e-6  # every workload is measured at residual 1e-6
