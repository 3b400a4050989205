"""Build librbm.so (HIP, gfx950) in-tree.

Each source is compiled to an object file in parallel (they are independent
translation units), then linked into one shared library.

Usage: python -m paper_1812_10575_amd.build   (or python paper_1812_10575_amd/build.py)
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librbm.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["rbm_kernels.hip", "rbm_cv.hip", "rbm_ensemble.hip", "rbm_rbmr.hip", "rbm_abi.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions: ordinary float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o")
        jobs.append((obj, [HIPCC] + FLAGS + ["-c", "-o", obj, os.path.join(CSRC, s)]))

    def run(job):
        if verbose:
            print(" ".join(job[1]), flush=True)
        subprocess.run(job[1], check=True)

    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        list(ex.map(run, jobs))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", OUT + ".tmp"] + [o for o, _ in jobs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
