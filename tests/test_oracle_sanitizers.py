"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code, gcc):
oracle/sanitize_driver.c calls every routine on small inputs; any out-of-bounds access, leak
or undefined operation aborts the run.  The same driver built without sanitizers gives the
same checksum (the sanitizers change nothing computed)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORA = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    srcs = [os.path.join(ORA, "sanitize_driver.c"), os.path.join(ORA, "sg_oracle.c")]
    base = ["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-I", ORA]
    san = str(tmp_path / "san")
    plain = str(tmp_path / "plain")
    subprocess.check_call(base + ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                  "-fno-omit-frame-pointer", *srcs, "-o", san, "-lm"])
    subprocess.check_call(base + [*srcs, "-o", plain, "-lm"])
    # verify_asan_link_order=0: the run is valid whatever else the environment preloads
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([san], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    p = subprocess.run([plain], capture_output=True, text=True, timeout=300, check=True)
    assert r.stdout == p.stdout and r.stdout.startswith("oracle checksum ")
