"""Build the gfx950 HIP library libbem_hip.so in-tree (hipcc, no JIT), and
the benchmark's small diagnostics library libbem_diag.so.

Run ``python -m paper_2312_12787_amd.build`` (or call ``build()``).  The
library exports the C ABI declared in include/bem.h.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbem_hip.so")
DIAG_LIB = os.path.join(HERE, "libbem_diag.so")  # streaming-read kernel of bench.py --mode peaks
SOURCES = ["assemble.hip", "linalg.hip", "matvec.hip", "nearfield.hip", "bem_api.cpp", "serve.cpp"]
ARCH = os.environ.get("BEM_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False, jobs: int = 4) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    common = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-result", "-pthread"]
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src + ".o")
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        cmd = [hipcc] + common + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    bad = [p.wait() for p in procs]
    if any(bad):
        raise RuntimeError("hipcc failed")
    link = [hipcc, "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    for o in objs:
        os.remove(o)
    diag = [hipcc] + common + ["-shared", os.path.join(CSRC, "diag.hip"), "-o", DIAG_LIB + ".tmp"]
    if verbose:
        print(" ".join(diag), flush=True)
    subprocess.run(diag, check=True)
    os.replace(DIAG_LIB + ".tmp", DIAG_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
