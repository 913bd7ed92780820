"""Compile the HIP sources into the in-tree shared library (gfx950).

Each translation unit is compiled to an object in parallel (every unit
carries its own device code object), then the objects are linked."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libsfft_mi355x.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 VALU forms stay disabled for every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs = jobs or min(len(sources()), max(1, len(os.sched_getaffinity(0))))
    with tempfile.TemporaryDirectory(prefix="sfft_build_") as tmpd:
        def compile_one(src):
            obj = os.path.join(tmpd, os.path.basename(src) + ".o")
            cmd = [hipcc, *HIPCC_FLAGS, *inc, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, capture_output=True, text=True)
            return obj, res
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(compile_one, sources()))
        bad = [r for _, r in results if r.returncode != 0]
        if bad:
            for r in bad:
                sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed compiling the SFFT library sources")
        tmp = OUT + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[o for o, _ in results]]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libsfft_mi355x.so")
        os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
