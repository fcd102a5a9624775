"""Builds libassg.so (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_1908_04081_amd.build`` or ``build()`` from Python.
Every call recompiles (objects go to paper_1908_04081_amd/_build/).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libassg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    f"-I{INCLUDE}", f"-I{CSRC}",
    # packed FP32 instructions stay off (this code is FP64; keep it explicit)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


def _compile(src, extra, objdir=BUILD):
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


DEBUG_LIB = os.path.join(PKG, "libassg_debug.so")
DEBUG_BUILD = os.path.join(PKG, "_build_debug")


def build(verbose: bool = False, extra=(), debug: bool = True) -> str:
    """Builds libassg.so and, unless ``debug`` is false, libassg_debug.so
    (the same sources with -DASSG_DEBUG: index checks in the kernels)."""
    lib = _build_lib(LIB, BUILD, list(extra), verbose)
    if debug:
        _build_lib(DEBUG_LIB, DEBUG_BUILD, [*extra, "-DASSG_DEBUG"], verbose)
    build_probe()
    build_example()
    return lib


def _build_lib(out: str, objdir: str, extra: list, verbose: bool) -> str:
    os.makedirs(objdir, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(lambda s: _compile(s, extra, objdir), srcs))
    if verbose:
        for obj, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *[o for o, _ in results]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


PROBE_DIR = os.path.join(PKG, "bwprobe")
PROBE_LIB = os.path.join(PROBE_DIR, "libassg_bwprobe.so")


def build_probe() -> str:
    """The bandwidth probes (paper_1908_04081_amd/bwprobe), a library of their
    own: measurement kernels, not part of the solver's ABI."""
    tmp = PROBE_LIB + ".tmp"
    cmd = [HIPCC, *COMMON, f"-I{PROBE_DIR}", "-shared", "-o", tmp,
           os.path.join(PROBE_DIR, "bwprobe.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for the bandwidth probes:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


EXAMPLE_SRC = os.path.join(PKG, "examples", "poisson2d.c")
EXAMPLE_BIN = os.path.join(PKG, "examples", "poisson2d")
CC = os.environ.get("CC", "gcc")


def example_cmd(out: str, extra=()) -> list:
    """Host compiler command for the plain C example (C11, the public header,
    linked against the built library and the HIP runtime)."""
    rocm = os.path.dirname(os.path.dirname(HIPCC)) if os.path.isabs(HIPCC) else "/opt/rocm"
    return [CC, "-O2", "-std=c11", "-Wall", "-Wextra", *extra, "-D__HIP_PLATFORM_AMD__",
            f"-I{rocm}/include", f"-I{INCLUDE}", EXAMPLE_SRC, "-o", out, f"-L{PKG}", "-lassg",
            f"-L{rocm}/lib", "-lamdhip64", "-lm", f"-Wl,-rpath,{PKG}"]


def build_example(out: str = EXAMPLE_BIN) -> str:
    r = subprocess.run(example_cmd(out), capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"C example failed to build:\n{r.stdout}\n{r.stderr}")
    return out


if __name__ == "__main__":
    print(build(verbose=True))
