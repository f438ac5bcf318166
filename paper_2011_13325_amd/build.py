"""Build libeamg.so (HIP kernels for gfx950 + host C++ setup + C ABI) in this directory.

Usage: python -m paper_2011_13325_amd.build   (or call build())
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libeamg.so")
ARCH = "gfx950"

HOST_SOURCES = ["coarsen.cpp", "structure.cpp", "api.cpp", "batch.cpp", "gnn_api.cpp",
                "staging.cpp", "fused.cpp"]
HIP_SOURCES = ["kernels.hip", "panel.hip", "gnn.hip", "coarse.hip", "criteria.hip", "noalloc.hip",
               "fused.hip"]
# the criteria must round like the host code (no fused multiply-add)
FILE_FLAGS = {"criteria.hip": ["-ffp-contract=off"]}

# Packed FP32 instructions are kept out of the device code (-packed-fp32-ops).
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=fast"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        jobs.append(([hipcc, *HIP_FLAGS, *FILE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj],
                     obj))
    for src in HOST_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        # host sources include the HIP runtime header: compile with hipcc in host-only mode
        jobs.append(([hipcc, *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for f in [ex.submit(_run, cmd, verbose) for cmd, _ in jobs]:
            f.result()
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd[:3])} ...")


if __name__ == "__main__":
    print(build(verbose=True))
