"""Builds libsched.so (all HIP sources for gfx950) in the package directory.

Each translation unit is compiled to an object of its own, in parallel, and
the objects are linked into one shared library; no device code calls across
translation units, so no relocatable device code is needed.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsched.so")
OBJ = os.path.join(PKG, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-mcode-object-version=5",
    # packed fp32 instructions stay off: plain float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = [l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l]
    return r.returncode, noise


def build(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(os.path.dirname(PKG), "include")]
    objs = [os.path.join(OBJ, os.path.basename(s)[:-4] + ".o") for s in srcs]
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_run, [hipcc(), *HIPCC_FLAGS, *inc, "-c", s, "-o", o], verbose)
                for s, o in zip(srcs, objs)]
        results = [f.result() for f in futs]
    failed = False
    for (rc, noise), s in zip(results, srcs):
        if noise and (rc != 0 or verbose):
            sys.stderr.write("\n".join(noise) + "\n")
        failed = failed or rc != 0
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    rc, noise = _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                     verbose)
    if rc != 0:
        sys.stderr.write("\n".join(noise) + "\n")
        raise RuntimeError(f"link failed ({rc})")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
