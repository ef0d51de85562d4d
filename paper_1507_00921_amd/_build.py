"""Build libdbp.so for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libdbp.so")
INCLUDE = os.path.join(ROOT, "include")

SOURCES = ["dbp.hip", "kern_small.hip", "kern_1024.hip", "kern_2048.hip", "kern_4096.hip",
           "kern_large.hip", "kern_fir.hip", "kern_mfma.hip",
           "kern_batch1.hip", "kern_batch2.hip", "batch.hip", "kern_adj1.hip", "kern_adj2.hip",
           "rx.hip", "kern_rx1.hip", "kern_rx2.hip", "rxdsp.hip", "mse.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++20", "--offload-arch=gfx950", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in [os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")]:
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))
    return res


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every translation unit (in parallel) and link lib/libdbp.so; always recompiles."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(LIBDIR, exist_ok=True)
    objdir = os.path.join(LIBDIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    jobs_list = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        jobs_list.append((obj, [cc, *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c",
                                os.path.join(CSRC, src), "-o", obj]))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda j: _run(j[1], verbose), jobs_list))
    tmp = LIB + ".tmp"
    _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in jobs_list], "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
