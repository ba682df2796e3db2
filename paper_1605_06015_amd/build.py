"""Build libbbx.so (HIP for gfx950) in-tree.

Each ``csrc/*.hip`` file is compiled by hipcc for gfx950 into an object under
``_build/``, then linked into ``paper_1605_06015_amd/libbbx.so``.  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libbbx.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


# The host code (argument validation, geometry preprocessing, slab bounds, ...) built
# with AddressSanitizer and UndefinedBehaviorSanitizer: each sanitizer flag applies to the
# host compilation only (device code is built as usual).  Loaded instead of libbbx.so
# when BBX_LIB names it; the process must preload clang's ASan runtime.
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
LIB_SAN = os.path.join(ROOT, "_build_asan", "libbbx_asan.so")
BUILD_SAN = os.path.join(ROOT, "_build_asan")


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(BUILD_SAN if sanitize else BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, *(SAN_FLAGS if sanitize else []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libbbx.so (always rebuilds); with
    sanitize, the sanitized host build libbbx_asan.so."""
    os.makedirs(BUILD_SAN if sanitize else BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, sanitize), srcs))
    lib = LIB_SAN if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


PROBE_SRC = os.path.join(PKG, "measure", "valu_issue_rate.hip")
PROBE = os.path.join(BUILD, "valu_issue_rate")


def build_probe(verbose: bool = False) -> str:
    """Compile the VALU issue-rate probe (a standalone measurement program behind the ALU
    roofline's slot costs, not part of the library) into _build/valu_issue_rate."""
    os.makedirs(BUILD, exist_ok=True)
    cmd = [HIPCC, "-O3", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Wall", "-o", PROBE, PROBE_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {PROBE_SRC}:\n{r.stdout}\n{r.stderr}")
    if verbose:
        print("built", PROBE)
    return PROBE


if __name__ == "__main__":
    if "--probe" in sys.argv:
        build_probe(verbose=True)
    else:
        build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)
