"""Build the HIP library ``libaprconv.so`` for gfx950 with hipcc.

Usage: ``python -m paper_2112_03592_amd.build`` (or ``build()``).  Always
recompiles: every source to an object file in parallel, then one link; the
output lands next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libaprconv.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-FP32 feature: drop that note
    err = "\n".join(ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln)
    return r.returncode, r.stdout + err


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    srcs = sources()
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 1), 16))
    with tempfile.TemporaryDirectory(prefix="aprconv_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.basename(s) + ".o") for s in srcs]
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            res = list(ex.map(lambda so: _run([hipcc, *HIPCC_FLAGS, *inc, "-c", so[0], "-o", so[1]], verbose),
                              zip(srcs, objs)))
        failed = [(s, out) for s, (rc, out) in zip(srcs, res) if rc != 0]
        for s, (rc, out) in zip(srcs, res):
            if out.strip() and (verbose or rc != 0):
                sys.stderr.write(f"--- {os.path.basename(s)}\n{out}\n")
        if failed:
            raise RuntimeError("hipcc failed on " + ", ".join(os.path.basename(s) for s, _ in failed))
        tmp = LIB + ".tmp"
        rc, out = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
        if rc != 0:
            sys.stderr.write(out)
            raise RuntimeError("hipcc failed linking libaprconv.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
