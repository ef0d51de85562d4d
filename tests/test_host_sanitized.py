"""The library's host code under AddressSanitizer, LeakSanitizer and UndefinedBehaviorSanitizer
(CPU only): a C++ driver calls every host path of the C ABI -- validation, FP64 schedule,
modelled and fixed geometry, FIR design, seeded fuzzing of descriptors, and the error paths
of the calls that need a device (there is none here) -- against a build whose host code is
instrumented (paper_1507_00921_amd/_build.py, build_sanitized)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_paths_under_sanitizers():
    if not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("the driver expects the device calls to fail: run where no GPU is visible")
    except ImportError:
        pass
    from paper_1507_00921_amd import _build
    driver = _build.build_sanitized()
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["LSAN_OPTIONS"] = "suppressions=" + os.path.join(ROOT, "tests", "sanitize", "lsan.supp")
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env.pop("LD_PRELOAD", None) if "asan" in env.get("LD_PRELOAD", "") else None
    r = subprocess.run([driver], env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert r.returncode == 0, out[-4000:]
    assert "checks passed" in r.stdout
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out
