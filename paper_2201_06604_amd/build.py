"""Build libmrg355.so (gfx950) in-tree with hipcc.

    python -m paper_2201_06604_amd.build
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmrg355.so")
SOURCES = ["mrg_kernels.hip", "mrg_tables.hip", "mrg_selfcheck.hip", "mrg_api.cpp", "mrg_batch.cpp",
           "mrg_server.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed-fp32 instructions stay off: hipcc would otherwise form them from
# ordinary float code.
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-fconstexpr-steps=100000000", "-ffp-contract=off",
             "-Wall", "-Wno-unused-result"]


def _compile(src, obj, extra=()):
    cmd = [HIPCC] + HIP_FLAGS + list(extra) + ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                               "-c", src, "-o", obj]
    subprocess.run(cmd, check=True, cwd=CSRC)


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link libmrg355.so."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(objdir, s + ".o")
        extra = [] if s.endswith(".hip") else ["-x", "hip"]
        if verbose:
            print("hipcc", s, flush=True)
        jobs.append((src, obj, extra))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "0")) or os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(_compile, *j) for j in jobs]:
            f.result()
    objs = [j[1] for j in jobs]
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs,
                   check=True, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
