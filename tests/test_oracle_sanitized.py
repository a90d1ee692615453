"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sanitize_check.c runs every entry point of the C oracle on small fixed
inputs (threads, empty and one-epoch lightcurves, a source on a lens, NaN and
infinite fitness, the largest population, rejected configurations).  It is
built twice from the same sources -- with the sanitizers and plainly -- and
both runs must end cleanly with identical output, which must also equal what
the ordinary oracle library computes from the printed inputs.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle")
SOURCES = [os.path.join(ORC, s) for s in ("sanitize_check.c", "sblm_oracle.c", "ea_oracle.c")]
BASE = ["gcc", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-pthread", "-Wall",
        "-Wextra"]
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]


def _build_and_run(tmp_path, name, flags):
    exe = str(tmp_path / name)
    subprocess.run(BASE + flags + SOURCES + ["-o", exe, "-lm"], check=True,
                   capture_output=True, text=True)
    # verify_asan_link_order=0: the environment may preload other libraries
    # ahead of the sanitizer runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23:"
               "verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)


def _parse(out):
    vals = {}
    for line in out.splitlines():
        parts = line.split()
        if len(parts) == 3:
            vals.setdefault(parts[0], {})[int(parts[1])] = float.fromhex(parts[2])
    return {k: np.array([v[i] for i in sorted(v)]) for k, v in vals.items()}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_sanitizers(tmp_path):
    san = _build_and_run(tmp_path, "check_san", SAN)
    assert "runtime error" not in san.stderr, san.stderr[-4000:]
    assert "AddressSanitizer" not in san.stderr, san.stderr[-4000:]
    assert "LeakSanitizer" not in san.stderr, san.stderr[-4000:]
    assert san.returncode == 0, san.stdout[-2000:] + san.stderr[-4000:]
    assert san.stdout.rstrip().endswith("fails 0")
    plain = _build_and_run(tmp_path, "check_plain", ["-O2"])
    assert plain.returncode == 0
    assert san.stdout == plain.stdout

    v = _parse(san.stdout)
    # the same computations through the ordinary oracle library
    th = v["mag_theta"].reshape(6, -1)
    A, ni = O.magnify(th, v["mag_t"], nthreads=1)
    assert np.array_equal(A.ravel(), v["mag_A"])
    assert np.array_equal(ni.ravel().astype(float), v["mag_nimg"])
    off = np.array([0, 0, 1, 24], dtype=np.int64)
    c2, fs, fb = O.chi2(off, v["chi_t"], v["chi_y"], v["chi_w"],
                        v["chi_theta"].reshape(6, -1), 3, nthreads=1)
    assert np.array_equal(c2, v["chi_chi2"])
    assert np.array_equal(fs, v["chi_Fs"]) and np.array_equal(fb, v["chi_Fb"])
    # the empty lightcurve fits nothing; the one-epoch one exactly
    assert np.all(c2[:3] == 0.0)
    assert np.all(np.abs(c2[3:6]) < 1e-20)
    # a source on a lens: the degree-4 polynomial still gives 3 images
    assert v["img_n"][0] == 3 and v["img_n"][1] == 3
    assert np.all(v["img_A"] >= 1.0)
