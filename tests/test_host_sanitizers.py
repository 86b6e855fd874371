"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

libsg is rebuilt with its host side instrumented (the device code is compiled as usual), and
tests/host_sanitize_driver.c calls every entry point whose work is host code: DSATUR, the
instance features, the ladder repair, and context creation for both methods with valid and
invalid configurations (without a GPU, a valid one builds every host table and stops at the
first device call).  Any out-of-bounds access, use after free, leak in the library or
undefined operation fails the run; the same driver linked against the ordinary build gives the
same checksum.  Runs only where no GPU is visible."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_10302_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"

pytestmark = pytest.mark.skipif(
    not (os.path.exists(HIPCC) and os.path.exists(CLANG)) or os.path.exists("/dev/kfd"),
    reason="needs hipcc and clang, and a machine without a visible GPU")

COMMON = ["--offload-arch=gfx950", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# host-side instrumentation only: every sanitizer flag applies to the host pass
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(args):
    subprocess.run(args, check=True, capture_output=True, text=True)


def test_library_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    objs = {}
    jobs = []
    for src, san in (("sg_kernels.hip", False), ("sg_mlp.hip", False), ("sg_api.cpp", True),
                     ("sg_mlp_api.cpp", True)):
        o = str(tmp_path / (src + ".o"))
        objs[src] = o
        jobs.append([HIPCC, *COMMON, "-O1", "-g", "-c", os.path.join(CSRC, src), "-o", o,
                     *(HOST_SAN if san else [])])
    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(_compile, jobs))
    lib_dir = tmp_path / "lib"
    lib_dir.mkdir()
    _compile([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs.values(), "-o",
              str(lib_dir / "libsg.so"), *HOST_SAN])
    driver = os.path.join(ROOT, "tests", "host_sanitize_driver.c")
    san = str(tmp_path / "san")
    plain = str(tmp_path / "plain")
    inc = ["-I", os.path.join(ROOT, "include")]
    _compile([CLANG, "-std=c11", "-O1", "-g", *inc, "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", driver, "-o", san,
              "-L", str(lib_dir), "-lsg", "-Wl,-rpath," + str(lib_dir), "-lm"])
    pkg = os.path.join(ROOT, "paper_2503_10302_amd")
    _compile([CLANG, "-std=c11", "-O1", *inc, driver, "-o", plain, "-L", pkg, "-lsg",
              "-Wl,-rpath," + pkg, "-lm"])
    supp = tmp_path / "lsan.supp"
    # leaks reported inside the HIP runtime's own start-up are not the library's
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libamd_comgr\n")
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               LSAN_OPTIONS=f"suppressions={supp}",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([san], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: " not in r.stderr, r.stderr[-4000:]
    p = subprocess.run([plain], capture_output=True, text=True, timeout=600, check=True)
    assert r.stdout == p.stdout and r.stdout.startswith("libsg host checksum "), (r.stdout, p.stdout)
