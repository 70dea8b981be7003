"""Build the gfx950 shared library ``librtproj.so`` from ``csrc/*.hip`` with hipcc.

Each source is compiled to its own object (in parallel, under ``_build/``),
then the objects are linked into the shared library."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librtproj.so")
OBJDIR = os.path.join(ROOT, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _filtered(text: str) -> str:
    return "\n".join(line for line in text.splitlines() if "packed-fp32-ops" not in line and line.strip())


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = os.path.join(OBJDIR, os.path.basename(src)[:-4] + ".o")
        res = subprocess.run([hipcc, *HIPCC_FLAGS, *inc, "-c", src, "-o", obj], capture_output=True, text=True)
        return src, obj, res

    jobs = jobs or min(len(srcs), max(1, len(os.sched_getaffinity(0))), 16)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(compile_one, srcs))
    msgs = []
    for src, _, res in results:
        text = _filtered(res.stdout + res.stderr)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(src)} ({res.returncode}):\n{text}")
        if text:
            msgs.append(text)
    tmp = LIB + ".tmp"
    res = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for _, o, _ in results], "-o", tmp],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed ({res.returncode}):\n{_filtered(res.stdout + res.stderr)}")
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
