"""The measurement script's command line, on the CPU: more than one GPU is
refused with a message (the evaluation runs on one GPU), and the oracle legs
it times report the host they ran on."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baselines_report_host_and_sample():
    sys.path.insert(0, ROOT)
    import bench
    import bz_inputs as gen
    f = gen.shock_batch(2, 16, 8.0, seed=2)
    plan = bench.oracle_plan(16, 6, 1.0)
    a = bench.cpu_baseline(f, 0.01, 16, 6, 1.0, "two N=16 cells", plan)
    b = bench.cpu_baseline_fft(f, 0.01, 16, 6, 1.0, "two N=16 cells", plan)
    for rec, kind in ((a, "oracle"), (b, "oracle_fft_threads")):
        assert rec["kind"] == kind and rec["unit"] == "cells*Q/s"
        assert rec["value"] > 0 and np.isfinite(rec["value"])
        assert rec["cores"] >= 1 and rec["nproc"] == os.cpu_count()
        assert rec["cpu"] and "two N=16 cells" in rec["sample"]
