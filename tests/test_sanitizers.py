"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer: the host side of the C-ABI's
sensor set-up (Alg. 1 tiling, ray mask and summed-area table, LiDAR units, argument checks) in
a small driver, and the oracle through every entry point from a child Python process."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _asan_runtime():
    r = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


pytestmark = pytest.mark.skipif(shutil.which("g++") is None or _asan_runtime() is None,
                                reason="needs g++ with the AddressSanitizer runtime")


def test_host_tables_under_sanitizers(tmp_path):
    exe = tmp_path / "host_tables_check"
    subprocess.run(["g++", "-std=c++17", "-O1", *SAN, "-I" + os.path.join(ROOT, "include"),
                    "-I" + os.path.join(ROOT, "paper_2510_12901_amd", "csrc"),
                    os.path.join(ROOT, "tests", "sanitize", "host_tables_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-4000:]


def test_oracle_under_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                    *SAN, os.path.join(ROOT, "oracle", "utoracle.cpp"), "-o", str(lib)], check=True)
    env = dict(os.environ, UTORACLE_LIB=str(lib), LD_PRELOAD=_asan_runtime(), OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize", "oracle_calls.py")], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-2000:], r.stderr[-4000:])
