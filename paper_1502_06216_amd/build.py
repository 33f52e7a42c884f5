"""Build libjko.so (HIP, gfx950) in the package directory.

    python -m paper_1502_06216_amd.build

Compiles every ``csrc/*.hip`` translation unit with hipcc for gfx950 (in
parallel) and links them into ``paper_1502_06216_amd/libjko.so``.  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libjko.so")
BUILD_DIR = os.path.join(PKG, "_build")

ARCH = "gfx950"
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC)")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(hipcc, src, obj, extra):
    cmd = [hipcc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c",
           "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}",
           *DEVICE_FLAGS, *extra, src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    return cmd, res


def build(verbose: bool = False, extra_flags=()) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(BUILD_DIR, os.path.basename(s)[:-4] + ".o") for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
        futs = [ex.submit(_compile, hipcc, s, o, list(extra_flags)) for s, o in zip(srcs, objs)]
        for f in futs:
            cmd, res = f.result()
            noise = [ln for ln in (res.stderr or "").splitlines()
                     if "packed-fp32-ops" not in ln]
            if res.returncode != 0:
                raise RuntimeError("compile failed:\n" + " ".join(cmd) + "\n" + "\n".join(noise))
            if verbose and noise:
                print("\n".join(noise), file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + " ".join(cmd) + "\n" + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
