"""Build the HIP library libr4d.so for gfx950, in the package directory.

    python paper_2402_03307_amd/build.py

Every source is compiled with hipcc for gfx950 (packed FP32 instructions
disabled) and linked into one shared library next to this file.  The same
objects also make abi_host_check, the C ABI's host-layer check
(tests/abi_host_check.cpp): the host layer (api.hip) compiled again with
AddressSanitizer and UndefinedBehaviorSanitizer on its host code only
(-Xarch_host), linked with the other objects as they are.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libr4d.so")
HOST_CHECK = os.path.join(PKG, "abi_host_check")
SOURCES = ("api.hip", "preprocess.hip", "binning.hip", "raster.hip", "consistency.hip",
           "training.hip")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC]


# host code only: no sanitizer reaches the device code
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
            "-fno-omit-frame-pointer"]


def _run(cmd, what):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{what} failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")


def build_host_check(verbose: bool = False) -> str:
    """abi_host_check from the objects of build() (which must have run)."""
    cc = hipcc()
    api = os.path.join(BUILD_DIR, "api_hostcheck.o")
    drv = os.path.join(BUILD_DIR, "abi_host_check.o")
    flags = [*compile_flags(), *SANITIZE, "-g"]
    flags[flags.index("-O3")] = "-O1"
    _run([cc, *flags, "-c", os.path.join(CSRC, "api.hip"), "-o", api], "compile")
    _run([cc, "-O1", "-g", "-std=c++17", *SANITIZE, "-I", INCLUDE, "-c",
          os.path.join(ROOT, "tests", "abi_host_check.cpp"), "-o", drv], "compile")
    others = [os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
              for src in SOURCES if src != "api.hip"]
    tmp = HOST_CHECK + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-g", *SANITIZE, "-o", tmp, drv, api, *others], "link")
    os.replace(tmp, HOST_CHECK)
    if verbose:
        print("linked", HOST_CHECK, flush=True)
    return HOST_CHECK


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()

    def one(src):
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [cc, *compile_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        if verbose:
            print("compiled", src, flush=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("linked", LIB, flush=True)
    build_host_check(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
