"""Build the gfx950 shared library ``libhd.so`` from ``csrc/`` with hipcc.

Every source is compiled for gfx950 only, with the packed-FP32 instructions
disabled (the compiler is asked not to form v_pk_* fp32 operations), and
linked into one shared library that exports the C ABI of include/hd.h.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhd.so")
SOURCES = ["k_cg.hip", "k_spmm.hip", "k_ugemm.hip", "k_ugemm_bf16.hip", "k_sparse_u.hip", "k_sim.hip", "k_topk.hip",
           "k_eig.hip", "hd_api.cpp", "hd_serve.cpp", "hd_tune.cpp", "hd_plan.cpp", "hd_planner.cpp", "hd_eig.cpp", "hd_fp8.cpp", "k_probe.hip", "k_persist.hip", "k_eig_gemm.hip", "hd_noalloc.hip"]
# ROCm libraries for the eigensolver's m x m steps (rocSOLVER: Cholesky and
# its inverse, the small symmetric eigenproblem; rocBLAS: its handle)
LIBS = ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-pthread", "-Wl,-rpath,/opt/rocm/lib"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build(verbose: bool = False) -> str:
    """Compile every source and link libhd.so (always rebuilds)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()

    def compile_one(src):
        obj = os.path.join(objdir, src + ".o")
        cmd = [cc] + flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
        p = subprocess.run(cmd, capture_output=True, text=True)
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{p.stderr}")
        if verbose:
            print("compiled", src, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + LIBS
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
