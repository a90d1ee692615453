"""bench.py's contract on the host (no GPU): the multi-GPU refusal, the peak
it divides by, and that its HBM-traffic figure belongs to the kernel source it
ships with."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    line = json.loads(res.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_fp64_vector_peak():
    # 256 compute units x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
    assert bench.PEAK_VALU_TFLOPS == pytest.approx(78.6432)


def test_traffic_figure_is_current():
    # the committed figure belongs to the committed kernel sources
    assert bench.fitness_traffic() == bench.FITNESS_TRAFFIC["bytes_per_launch"]


def test_traffic_figure_matches_the_kernel_source():
    # the committed rocprofv3 traffic is reported only for the source it was
    # measured on; for a changed kernel the bench reports null until it is
    # profiled again
    import hashlib
    h = hashlib.sha256()
    for f in ("sblm_fitness.hip", "sblm_math.h", "sblm_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1208_4830_amd", "csrc", f), "rb").read())
    want = bench.FITNESS_TRAFFIC["bytes_per_launch"] \
        if h.hexdigest()[:16] == bench.FITNESS_TRAFFIC["source_sha256_16"] else None
    assert bench.fitness_traffic() == want
    assert bench.FITNESS_TRAFFIC["bytes_per_launch"] > \
        bench.FITNESS_TRAFFIC["algorithmic_bytes_per_launch"]
