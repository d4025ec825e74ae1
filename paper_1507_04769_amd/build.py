"""Build libsgcm.so (gfx950) in-tree with hipcc.

Usage: python -m paper_1507_04769_amd.build   (or import and call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsgcm.so")
SOURCES = ["grid.cpp", "capi.cpp", "bvp.hip", "first_steps.hip", "example3.hip", "lobatto.hip", "interp.hip", "validate.hip"]
ARCH = os.environ.get("SGCM_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def _stale(obj: str, src: str, headers: list) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src] + headers)


def build(verbose: bool = False, jobs: int = 4, incremental: bool = False) -> str:
    """Compile every source to an object in parallel, then link the library.
    incremental: recompile only the sources (or headers) newer than their
    objects."""
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    hipcc = _hipcc()
    common = ["-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
              "-Wall"]
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers.append(os.path.join(ROOT, "include", "sgcm.h"))
    procs, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(obj_dir, src + ".o")
        objs.append(obj)
        if incremental and not _stale(obj, path, headers):
            continue
        if src.endswith(".hip"):
            cmd = [hipcc, "-x", "hip", "--offload-arch=" + ARCH] + DEVICE_FLAGS + common + ["-c", path,
                                                                                             "-o", obj]
        else:
            cmd = [hipcc, "-x", "c++", "-D__HIP_PLATFORM_AMD__"] + common + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[[i for i, (_, p) in enumerate(procs) if p.poll() is None][0]][1].wait()
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, out))
        elif verbose and out.strip():
            print(out)
    if failed:
        msg = "\n".join("== %s ==\n%s" % f for f in failed)
        raise RuntimeError("libsgcm build failed:\n" + msg)
    tmp = LIB + ".tmp%d" % os.getpid()
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L" + rocm_lib, "-Wl,-rpath," + rocm_lib, "-lrocprofiler-sdk-roctx"]  # roctx ranges of the C-ABI calls
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
