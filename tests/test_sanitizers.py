"""The oracle and the library's host-side code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): oracle.c built by gcc with both, and the
library's host code built by hipcc with both (device code is not
instrumented), each loaded into a fresh Python process with its sanitizer
runtime preloaded, which then runs the oracle's pins and the C-ABI host
checks.  Any report ends that process with an error."""
import glob
import os
import subprocess
import sys

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _run(env_extra, args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4", **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider", "-p", "no:xdist",
                        *args], env=env, cwd=REPO, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr


def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", *SAN_FLAGS,
                    os.path.join(REPO, "oracle", "oracle.c"), "-o", lib, "-lm"], check=True)
    rt = [subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
          for n in ("libasan.so", "libubsan.so")]
    _run({"LD_PRELOAD": ":".join(rt), "B2SR_ORACLE_LIB": lib}, ["tests/test_oracle.py"])


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2201_08560_amd import build_lib
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts:
        pytest.skip("no clang AddressSanitizer runtime")
    flags = []
    for f in SAN_FLAGS:  # host code only: each sanitizer flag behind -Xarch_host
        flags += ["-Xarch_host", f]
    lib = build_lib.build(extra_flags=flags, out=str(tmp_path / "libb2sr_san.so"))
    _run({"LD_PRELOAD": rts[0], "B2SR_LIB": lib}, ["tests/test_abi.py", "tests/test_serve.py"])
