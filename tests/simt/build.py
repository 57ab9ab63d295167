"""Builds the graph sweep and the job readiness sweep (graph.hip, jobs.hip
and the host code of libllp) against the
CPU emulation in tests/simt/hip/hip_runtime.h into tests/simt/_build/
libllp_simt.so, with AddressSanitizer when the host compiler has it.  Test
infrastructure only: the product library is built by paper_2603_13147_amd/_build.py."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2603_13147_amd", "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "libllp_simt.so")
SOURCES = [os.path.join(CSRC, f) for f in ("graph.hip", "jobs.hip", "llp_host.cpp", "sched_host.cpp", "abi.cpp", "tune.cpp")] + \
          [os.path.join(HERE, f) for f in ("simt.cpp", "stubs.cpp")]


def asan_runtime():
    """Path of the host compiler's AddressSanitizer runtime, or None."""
    r = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    san = ["-fsanitize=address", "-fno-omit-frame-pointer"] if asan_runtime() else []
    flags = ["-std=c++17", "-O1", "-g", "-fPIC", "-I", HERE, "-Wno-unused-result", "-Wno-attributes", *san]
    # objects and the unlinked library are private to this process, so test
    # workers that build at the same time do not overwrite each other's files
    # (the finished library replaces the old one in a single rename)
    odir = os.path.join(OUT, f"obj-{os.getpid()}")
    os.makedirs(odir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(odir, os.path.basename(src) + ".o")
        lang = ["-x", "c++"] if src.endswith(".hip") else []
        r = subprocess.run(["g++", *flags, *lang, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"g++ failed for {src}:\n{r.stderr}")
        objs.append(obj)
    tmp = LIB + f".{os.getpid()}.tmp"
    r = subprocess.run(["g++", *san, "-shared", "-o", tmp, *objs], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    shutil.rmtree(odir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build())
