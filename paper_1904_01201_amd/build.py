"""Build libhabmi.so (HIP kernels + host runtime + C ABI) for gfx950.

Usage: python -m paper_1904_01201_amd.build [--jobs N] [--sanitize]

--sanitize builds _build_san/libhabmi_san.so instead: the same sources with the host
code instrumented by AddressSanitizer and UndefinedBehaviorSanitizer (the
device code is built as usual), for CPU tests of the host runtime; it is
loaded with the compiler's ASan runtime preloaded.

Every source is compiled by hipcc with contraction off (the rendering
arithmetic is specified operation by operation) and packed fp32 ops
disabled, then linked into one shared library next to this file.
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libhabmi.so")
OBJDIR = os.path.join(HERE, "_build")
SAN_OBJDIR = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_OBJDIR, "libhabmi_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all", "-g"]
SOURCES = ["kernels.hip", "actuate.hip", "noalloc.hip", "runtime.cpp", "abi.cpp", "stepper.cpp",
           "server.cpp", "autotune.cpp"]
ARCH = os.environ.get("HABMI_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(SAN_OBJDIR if sanitize else OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *(SAN_FLAGS if sanitize else [])]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msgs}")
    if msgs.strip():
        print(msgs, file=sys.stderr)
    return obj


def build(jobs: int = 6, sanitize: bool = False) -> str:
    """Compile and link; always rebuilds."""
    objdir, lib = (SAN_OBJDIR, SAN_LIB) if sanitize else (OBJDIR, LIB)
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), srcs))
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--sanitize", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.sanitize))
