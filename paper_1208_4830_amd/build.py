"""Builds libsblm.so (all HIP sources of csrc/) for gfx950, in-tree.

Each source is compiled to an object of its own, in parallel (no device code
crosses translation units: kernels are launched by host functions of their
own file), then the objects are linked into the shared library.
"""
import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsblm.so")
OBJDIR = os.path.join(os.path.dirname(HERE), "_build", "libsblm")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no implicit contraction: every fused multiply-add is written as fma()
    "-ffp-contract=off",
    # packed FP32 instructions are not emitted
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _filter(stderr):
    return "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l)


def build(verbose: bool = False, extra_flags=(), lib=LIB) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    tag = "" if lib == LIB else "_" + os.path.basename(lib).replace(".", "_")
    jobs = []
    for src in sources():
        obj = os.path.join(OBJDIR, os.path.basename(src)[:-4] + tag + ".o")
        jobs.append((src, obj, [hipcc] + HIPCC_FLAGS + list(extra_flags) + ["-c", src, "-o", obj]))

    def run(job):
        src, obj, cmd = job
        if verbose:
            print(" ".join(cmd), flush=True)
        return src, subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        results = list(ex.map(run, jobs))
    for src, res in results:
        err = _filter(res.stderr)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n" + err)
        if verbose and err.strip():
            print(err)
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for _, o, _ in jobs] + \
        ["-o", lib + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + _filter(res.stderr))
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
