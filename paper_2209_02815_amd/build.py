"""Compile the HIP library libh1w.so in-tree for gfx950 (MI355X).

Every .hip file under csrc/ is compiled by hipcc to an object in _build/
(in parallel) and linked into paper_2209_02815_amd/libh1w.so. Packed FP32
instructions are disabled for all device code.
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
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libh1w.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


# host-code AddressSanitizer build (device code is built as usual): for CPU
# tests of the host paths (argument validation, error handling) under ASan
ASAN_LIB = os.path.join(PKG, "libh1w_asan.so")
ASAN_FLAGS = ["-O1", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, asan: bool = False) -> str:
    out = os.path.join(BUILD, "asan") if asan else BUILD
    obj = os.path.join(out, os.path.basename(src) + ".o")
    flags = [f for f in CFLAGS if f != "-O3"] + ASAN_FLAGS if asan else CFLAGS
    cmd = [HIPCC, *flags, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if err:
        print(err, file=sys.stderr)
    return obj


def build(jobs: int | None = None, asan: bool = False) -> str:
    """Compile and link libh1w.so (or, with asan, libh1w_asan.so: host code
    instrumented by AddressSanitizer, whose runtime the loading process must
    preload)."""
    os.makedirs(os.path.join(BUILD, "asan") if asan else BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, asan), srcs))
    lib = ASAN_LIB if asan else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(asan="--asan" in sys.argv[1:]))
