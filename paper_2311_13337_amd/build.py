"""Builds libvadx.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Packed FP32 instructions are switched off for all device code
(-target-feature -packed-fp32-ops); the host pass warns that it does not know
the feature, which is harmless.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvadx.so")
SOURCES = [os.path.join(CSRC, f) for f in ("kernels.hip", "vadx_api.cpp", "mlp.hip", "mlp_api.cpp", "select.hip",
                                              "analysis.hip", "analysis_api.cpp", "bold.hip")]
HOST_SOURCES = [os.path.join(CSRC, "opcount.cpp")]   # plain C++ (g++), no device code
ARCH = os.environ.get("VADX_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _compile(cmd: list, src: str, what: str) -> str:
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"{what} failed on {src}")
    return r.stderr


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compiles every source (in parallel, `jobs` processes, default one per
    source up to the host's cores) and links libvadx.so (always rebuilds)."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    work = []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        work.append(([hipcc(), *common, *lang, "-c", src, "-o", obj], src, "hipcc", obj))
    for src in HOST_SOURCES:
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        work.append((["g++", "-O2", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                      "-c", src, "-o", obj], src, "g++", obj))
    n = jobs or max(1, min(len(work), os.cpu_count() or 1, 16))
    with concurrent.futures.ThreadPoolExecutor(max_workers=n) as pool:
        futs = [pool.submit(_compile, cmd, src, what) for cmd, src, what, _ in work]
        for f in futs:
            log = f.result()
            if verbose:
                sys.stderr.write(log)
    objs = [obj for *_, obj in work]
    tmp = LIB + ".tmp"
    r = subprocess.run([hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libvadx.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
