"""Build the HIP library (libfds.so) in-tree for gfx950.

Every source under csrc/ is compiled with hipcc; kernels.hip is the only
translation unit with device code.  Packed-FP32 instructions are disabled for
device code."""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
# FDS_BUILD_OUT / FDS_BUILD_DIR / FDS_BUILD_DEFINES (development only) build a
# variant library elsewhere, e.g. with -DFDS_HANDOFF_FENCED
OUT = os.environ.get("FDS_BUILD_OUT", os.path.join(HERE, "libfds.so"))
BUILD_DIR = os.environ.get("FDS_BUILD_DIR", os.path.join(ROOT, "_build"))
DEFINES = os.environ.get("FDS_BUILD_DEFINES", "").split()

SOURCES = ["kernels.hip", "dst_wave.hip", "ik_kernels.hip", "alloc.cpp", "tune.cpp", "tables.cpp", "plan.cpp", "engine.cpp", "server.cpp", "abi.cpp"]
ARCH = os.environ.get("FDS_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags(src: str):
    f = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", *DEFINES]
    if src.endswith(".hip"):
        f += ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]
    else:
        f += ["-D__HIP_PLATFORM_AMD__"]
    return f


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    objs = []

    # FDS_BUILD_INCREMENTAL=1 (development only): keep objects newer than
    # their source and every header; the default rebuilds everything
    incremental = os.environ.get("FDS_BUILD_INCREMENTAL") == "1"
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers.append(os.path.join(ROOT, "include", "fds.h"))
    newest_header = max(os.path.getmtime(h) for h in headers)

    def compile_one(src):
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        if incremental and os.path.exists(obj):
            t = os.path.getmtime(obj)
            if t > os.path.getmtime(os.path.join(CSRC, src)) and t > newest_header:
                return obj
        cmd = [cc, *_flags(src), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
