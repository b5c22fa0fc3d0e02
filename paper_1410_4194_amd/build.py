"""Build the HIP library ``libctu.so`` for gfx950 in-tree.

Usage: ``python -m paper_1410_4194_amd.build`` (or via ``__graft_entry__.build()``).
Packed FP32 instructions are disabled for all device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libctu.so")
ARCH = os.environ.get("CTU_OFFLOAD_ARCH", "gfx950")
# (source, object, extra defines): the sweep kernels are compiled once per storage type,
# solver class (exact solver per gas class 0, 3, 5; Roe solver 1; Roe with the H correction
# 2) and reconstruction (PPMC 0, PPMP 1), in parallel
UNITS = [("ctu_kernels.hip", "ctu_kernels.o", []), ("ctu_runtime.cpp", "ctu_runtime.o", []),
         ("ctu_stream.hip", "ctu_stream.o", [])] + [
    ("ctu_sweeps.hip", f"ctu_sweeps_{t[0]}{k}{'p' if r else ''}.o",
     [f"-DCTU_SWEEP_T={t}", f"-DCTU_SWEEP_K={k}", f"-DCTU_SWEEP_R={r}"])
    for t in ("double", "float") for k in (0, 1, 2, 3, 5) for r in (0, 1)]


def build(verbose: bool = False, jobs: int = 0) -> str:
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmds, objs = [], []
    for src, obj, defs in UNITS:
        obj = os.path.join(CSRC, obj)
        cmds.append([hipcc, "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                     "-Wall", "-Wno-unused-function", *defs,
                     "-I", os.path.join(REPO, "include"), "-I", CSRC,
                     "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(run, c) for c in cmds]:
            f.result()
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    for obj in objs:
        os.remove(obj)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
