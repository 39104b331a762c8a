"""Build libmcspect.so for gfx950 with hipcc (cross-compiles without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmcspect.so")
# issue-rate probes for the benchmark's roofline (not part of the product library)
PROBE_LIB = os.path.join(HERE, "libmcprobe.so")
# measurement build: the same sources with the transport loop's region markers
# (MC_REGION_PROFILE), loaded only by region_profile.py
PROF_LIB = os.path.join(HERE, "libmcspect_prof.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["api.hip", "staging.hip", "transport.hip", "adjoint.hip", "sysmat.hip", "cfd.hip", "cgsm.hip",
           "compose.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def compile_one(src: str, profile: bool = False) -> str:
    out_dir = BUILD_DIR + ("_prof" if profile else "")
    os.makedirs(out_dir, exist_ok=True)
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *HIPCC_FLAGS, *(["-DMC_REGION_PROFILE"] if profile else []), "-I", INCLUDE, "-I", CSRC,
           "-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.check_call(cmd)
    return obj


def _link(objs, lib: str) -> None:
    tmp = lib + ".tmp"
    subprocess.check_call([_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp])
    os.replace(tmp, lib)


def build_profile(verbose: bool = False) -> str:
    """The measurement build (region markers in the transport loop)."""
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 4)) as ex:
        objs = list(ex.map(lambda src: compile_one(src, True), SOURCES))
    _link(objs, PROF_LIB)
    if verbose:
        print("built", PROF_LIB)
    return PROF_LIB


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link the shared library (always rebuilds)."""
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 4)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    _link(objs, LIB)
    probe = compile_one("probe.hip")
    subprocess.check_call([_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", probe, "-o",
                           PROBE_LIB + ".tmp"])
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    if "--profile" in sys.argv:
        build_profile(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
