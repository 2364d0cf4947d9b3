"""Build libfrmi.so (HIP kernels for gfx950 + host construction + C ABI) in-tree.

Usage: python -m paper_2312_14167_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfrmi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("FRMI_ARCH", "gfx950")

SOURCES = ["fr_host.cpp", "fr_stats.cpp", "fr_kernels.hip", "fr_vjp.hip", "fr_geo.hip", "fr_vardeg.hip", "fr_api.hip"]
CLANG = os.environ.get("FRMI_CLANG", "/opt/rocm/lib/llvm/bin/clang++")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
          "-I", os.path.join(ROOT, "include"),
          # packed-FP32 VALU forms are kept out of the generated code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def _torch_hip_dir() -> str:
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or spec.origin is None:
        raise RuntimeError("PyTorch (ROCm) is required: its HIP runtime is the one the library links")
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so under {d}")
    return d


def _compile(src: str, outdir: str) -> str:
    obj = os.path.join(outdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    outdir = os.path.join(PKG, "_build")
    os.makedirs(outdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, outdir), SOURCES))
    tmp = LIB + ".tmp"
    # Link against the HIP runtime that PyTorch itself loads, so device pointers and streams handed
    # over by torch belong to the same runtime instance as our launches.
    hip_dir = _torch_hip_dir()
    cmd = [CLANG, "-shared", "-fPIC", "-o", tmp, *objs, f"-L{hip_dir}", "-l:libamdhip64.so",
           f"-Wl,-rpath,{hip_dir}", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
