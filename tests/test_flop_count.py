"""The FLOP counts behind the roofline come from the kernel's own arithmetic:
paper_1208_4830_amd/csrc/flop_count.cpp instantiates the shared code of
sblm_math.h (the code the fitness kernel runs) with a number type that counts
its operations.  The bench's per-call constants must equal that count, so a
change of the arithmetic cannot leave the roofline numerator stale."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

CSRC = os.path.join(ROOT, "paper_1208_4830_amd", "csrc")


@pytest.fixture(scope="module")
def counts(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("flops") / "flop_count")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wno-unknown-pragmas", "-I", CSRC,
                    os.path.join(CSRC, "flop_count.cpp"), "-o", exe], check=True)
    return json.loads(subprocess.run([exe], check=True, capture_output=True,
                                     text=True).stdout)


def test_bench_constants_are_the_counted_ones(counts):
    assert bench.FLOP_COUNTS == counts


def test_counts_are_consistent(counts):
    # an FP32 sweep skips the reciprocal refinement of the FP64 one; the
    # two-step refinement evaluates the lens equation once more than the
    # one-step one; the counts are those of straight-line code (no branch of
    # the counted paths is data dependent beyond the stated cases)
    assert counts["sweep32"] < counts["sweep64"]
    assert counts["refine"] - counts["refine1"] > counts["eval"]
    # one sweep: 10 pairwise reciprocals and five Horner evaluations of p and
    # p' (9 complex multiply-adds of 8 FLOPs each) at least
    assert counts["sweep64"] > 5 * 9 * 8 + 10 * 3
    per_mag = bench.flop_per_magnification(sweeps64=1.0, sweeps32=0.0, refined=0.0)
    assert per_mag == (counts["coef"] + counts["warm"] + counts["sweep64"] + counts["images"]
                       + counts["lsq"])
