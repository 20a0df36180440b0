"""Build libbsi.so (HIP kernels + C ABI) for gfx950 with hipcc.

Usage: python -m paper_2604_22048_amd.build   (or call build())
Objects are compiled in parallel into paper_2604_22048_amd/_build/ and linked
into paper_2604_22048_amd/libbsi.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libbsi.so")
SOURCES = ["transform.hip", "dft_mfma.hip", "likelihood.hip", "hmc.hip", "shear.hip", "bootstrap.hip",
           "diag.hip", "slots.hip", "stage.hip", "api.cpp",
           "slots.cpp", "autotune.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions are kept out of every kernel on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-command-line-argument",
    # lifetime mistakes (a returned temporary, a dangling reference) stop the build
    "-Werror=return-stack-address", "-Werror=dangling",
]


def _compile(src: str, bdir: str, defines=()) -> str:
    obj = os.path.join(bdir, src.replace(".", "_") + ".o")
    cmd = [HIPCC, *FLAGS, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, out: str = OUT, bdir: str | None = None, defines=()) -> str:
    """Compile every source and link `out`; `defines` are extra -D macros."""
    bdir = bdir or os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(lambda s: _compile(s, bdir, defines), SOURCES))
    tmp = out + ".tmp"
    r = subprocess.run([HIPCC, "-shared", "--offload-arch=gfx950", "-Wl,-z,defs", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
