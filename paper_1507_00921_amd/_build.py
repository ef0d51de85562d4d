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
           "rx.hip", "kern_rx1.hip", "kern_rx2.hip", "rxdsp.hip", "mse.hip", "kern_persist.hip",
           "kern_each.hip", "kern_keep1.hip", "kern_keep2.hip"]

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


# Host code (planner, schedule, geometry, FIR design, handles and their error paths) checked
# by AddressSanitizer and UndefinedBehaviorSanitizer: these translation units get the
# sanitizers on their host pass only (-Xarch_host before every host-only flag; the GPU code is
# compiled as usual), the kernel-only units are taken from the regular build.
SANITIZED = ["dbp.hip", "batch.hip", "rx.hip", "rxdsp.hip", "mse.hip"]
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-g"]
SANDIR = os.path.join(LIBDIR, "san")
DRIVER_SRC = os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")


def _sources_hash(extra=()):
    import hashlib
    h = hashlib.sha256()
    names = sorted(os.listdir(CSRC))
    for n in names:
        with open(os.path.join(CSRC, n), "rb") as f:
            h.update(n.encode() + f.read())
    for path in [os.path.join(INCLUDE, "dbp.h"), DRIVER_SRC, *extra]:
        with open(path, "rb") as f:
            h.update(f.read())
    h.update(" ".join(HIPCC_FLAGS + SAN_FLAGS).encode())
    return h.hexdigest()


def build_sanitized(verbose: bool = False, jobs: int = 8) -> str:
    """Build lib/san/libdbp_san.so (host code sanitized) and the host driver that exercises it;
    returns the driver's path.  Rebuilt only when a source changed."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(SANDIR, exist_ok=True)
    driver = os.path.join(SANDIR, "host_driver")
    stamp = os.path.join(SANDIR, "stamp")
    digest = _sources_hash()
    if os.path.exists(driver) and os.path.exists(stamp) and open(stamp).read() == digest:
        return driver
    cc = hipcc()
    objdir = os.path.join(SANDIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    jobs_list = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        flags = HIPCC_FLAGS + (SAN_FLAGS if src in SANITIZED else [])
        jobs_list.append((obj, [cc, *flags, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda j: _run(j[1], verbose), jobs_list))
    lib = os.path.join(SANDIR, "libdbp_san.so")
    _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in jobs_list], "-o", lib], verbose)
    clangxx = os.path.join(os.path.dirname(cc), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clangxx):
        clangxx = "/opt/rocm/llvm/bin/clang++"
    _run([clangxx, "-std=c++17", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", "-I", INCLUDE, DRIVER_SRC, "-L", SANDIR, "-ldbp_san",
          "-Wl,-rpath," + SANDIR, "-o", driver], verbose)
    with open(stamp, "w") as f:
        f.write(digest)
    return driver


if __name__ == "__main__":
    print(build(verbose=True))
