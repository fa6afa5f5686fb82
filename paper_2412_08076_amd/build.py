"""Build librm.so (HIP, gfx950) in place next to this file.

    python -m paper_2412_08076_amd.build

Compiles every HIP source under csrc/ with hipcc for gfx950 only.  Packed FP32
instructions are disabled (``-packed-fp32-ops``); the host pass of hipcc warns
that it does not know that target feature, which is harmless.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librm.so")
# the longest compiles first, so that they start at once
SOURCES = ["rm_stream.hip", "rm_mixed.hip", "rm_block.hip", "rm_kernels.hip", "rm_ssor.hip", "rm_twogrid.hip",
           "rm_symbolnet.hip", "rm_krylov.hip", "rm_api.hip"]
ARCH = "gfx950"


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ]


def build(verbose=False, jobs=None):
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    objs = [os.path.join(build_dir, src.replace(".hip", ".o")) for src in SOURCES]

    def compile_one(k):
        cmd = [hipcc()] + flags() + ["-c", os.path.join(CSRC, SOURCES[k]), "-o", objs[k]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    # one hipcc per source, at most one per host core (each takes one core)
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        list(pool.map(compile_one, range(len(SOURCES))))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
