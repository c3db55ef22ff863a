"""The oracle's C sweep under AddressSanitizer and UndefinedBehaviorSanitizer: rt_oracle.c
is built with both (every report fatal) and the oracle's pin tests run against that
build in a child process.  An out-of-bounds read or write, a use of freed memory or
undefined arithmetic anywhere on those paths (periodic, fixed and cold ghosts, both
orders, the quadratic upwind intensity, Gauss-Seidel) fails this test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def _asan_runtime():
    try:
        path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_tests_pass_under_sanitizers(tmp_path):
    preload = os.environ.get("LD_PRELOAD", "")
    system_preload = os.path.exists("/etc/ld.so.preload") and open("/etc/ld.so.preload").read().strip()
    if preload or system_preload:
        pytest.skip("another library is preloaded; the sanitizer runtime must come first")
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "rt_oracle_sanitized.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-o", lib, os.path.join(ROOT, "oracle", "rt_oracle.c"), "-lm"])
    tests = sorted(f for f in glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py"))
                   if not f.endswith("test_oracle_sanitized.py"))
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", RTSC_ORACLE_LIB=lib)
    probe = subprocess.run([sys.executable, "-c", "import oracle; oracle._load(); print(oracle._lib._name)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0 and probe.stdout.strip() == lib, probe.stderr[-2000:]
    # --capture=sys leaves file descriptor 2 alone, so a sanitizer report reaches stderr
    run = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "--capture=sys",
                          "-m", "not gpu", *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = run.stdout[-3000:] + run.stderr[-3000:]
    assert run.returncode == 0, out
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, out
