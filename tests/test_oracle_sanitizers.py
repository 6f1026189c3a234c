"""The FP64 oracle built with AddressSanitizer, UndefinedBehaviorSanitizer and
LeakSanitizer, driven through every entry point on a small procedural scene
(tests/sanitize/oracle_driver.c): any out-of-bounds access, use after free,
leak, signed overflow, misaligned access or other undefined behaviour fails
the test.  CPU only."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")
ORACLE = os.path.join(ROOT, "oracle", "bz_oracle.c")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_address_and_undefined_sanitizers():
    tmp = tempfile.mkdtemp(prefix="orc_san_")
    try:
        exe = os.path.join(tmp, "oracle_driver")
        cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               DRIVER, ORACLE, "-o", exe, "-lm"]
        subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        report = r.stdout + r.stderr
        assert r.returncode == 0, report
        assert "runtime error" not in report and "AddressSanitizer" not in report, report
        assert "LeakSanitizer" not in report, report
        assert "contributing pairs" in r.stdout
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
