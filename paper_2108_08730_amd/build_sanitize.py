"""Host-sanitizer builds of libhelm27 for CPU-side testing.

``python -m paper_2108_08730_amd.build_sanitize [address|thread]`` compiles
the library's host sources (table build, operator set-up, solver and serving
host logic) with AddressSanitizer + UndefinedBehaviorSanitizer ("address")
or ThreadSanitizer ("thread"), host code only, and links them with the
kernel objects of the regular build (``build.py``, which must have run).
The result, ``libhelm27_asan.so`` / ``libhelm27_tsan.so`` in the build
folder (``lib_path``), is loaded by setting HELM27_LIB to its path and preloading
the matching sanitizer runtime (``runtime_path``); ``tests/test_host_sanitize.py``
runs the host-library tests that way.  These builds are for the CPU: they
are never used for GPU runs.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

from . import build as B

HOST_SOURCES = ["table.cpp", "op.cpp", "solver.cpp", "serve.cpp"]
FLAGS = {
    "address": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"],
    "thread": ["-Xarch_host", "-fsanitize=thread"],
}
RUNTIME = {"address": "libclang_rt.asan-x86_64.so", "thread": "libclang_rt.tsan-x86_64.so"}


def lib_path(kind: str) -> str:
    return os.path.join(B.BUILD, "san_" + kind, "libhelm27_asan.so" if kind == "address" else "libhelm27_tsan.so")


def runtime_path(kind: str) -> str:
    hits = sorted(glob.glob(f"/opt/rocm/llvm/lib/clang/*/lib/linux/{RUNTIME[kind]}"))
    if not hits:
        raise RuntimeError(f"{RUNTIME[kind]} not found under /opt/rocm/llvm")
    return hits[-1]


def build(kind: str = "address") -> str:
    out_dir = os.path.join(B.BUILD, "san_" + kind)
    os.makedirs(out_dir, exist_ok=True)
    kernel_objs = [os.path.join(B.BUILD, s + ".o") for s in B.SOURCES if s.endswith(".hip")]
    missing = [o for o in kernel_objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"run the regular build first (missing {missing[0]})")
    san = FLAGS[kind]

    def comp(src):
        obj = os.path.join(out_dir, src + ".o")
        cmd = [B.HIPCC, "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}",
               "--offload-host-only", "-ffp-contract=off", "-I", B.INCLUDE, "-I", B.CSRC,
               "-Xarch_host", "-fno-omit-frame-pointer", *san, "-c", os.path.join(B.CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitizer build failed for {src}:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=len(HOST_SOURCES)) as ex:
        objs = list(ex.map(comp, HOST_SOURCES))
    lib = lib_path(kind)
    cmd = [B.HIPCC, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", *objs, *kernel_objs, *san, "-shared-libsan",
           "-o", lib]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitizer link failed:\n{r.stderr}")
    return lib


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else "address"))
