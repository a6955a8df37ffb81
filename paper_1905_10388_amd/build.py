"""Build the HIP library libstau.so in-tree for gfx950 (hipcc)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libstau.so")
# the check build: the same sources with the kernels' index checks compiled in
# (STAU_CHECK_BOUNDS, reported by stau_check)
LIB_CHECK = os.path.join(PKG, "libstau_check.so")
SOURCES = ["stau.hip", "k_pencil.hip", "k_factor.hip", "k_evp.hip", "k_transform.hip", "k_xpass.hip",
           "k_adjoint.hip", "k_dctmm.hip", "k_grid.hip"]
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed-FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def build(verbose: bool = False, check: bool = False) -> str:
    """Compile every source and link libstau.so (check=True: libstau_check.so
    with the index checks)."""
    objdir = os.path.join(PKG, "_build_check" if check else "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    flags = FLAGS + (["-DSTAU_CHECK_BOUNDS"] if check else [])
    lib = LIB_CHECK if check else LIB

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [cc, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = lib + ".tmp"
    cmd = [cc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, check="--check" in sys.argv))
