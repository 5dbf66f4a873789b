"""The oracle's pin suite against an AddressSanitizer + UndefinedBehavior-
Sanitizer build of oracle/oracle.c (CPU only).

The C oracle is built with -fsanitize=address,undefined and
-fno-sanitize-recover, loaded by a fresh Python process with the sanitizer
runtimes preloaded, and the pin files run against it: any out-of-bounds
access, use after free or undefined operation (signed overflow, a shift out
of range, a misaligned access) aborts that process and fails this test.  Two
long multi-thousand-step runs are left out; shorter pins exercise the same
code paths.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PIN_FILES = ["tests/test_oracle_step.py", "tests/test_oracle_adjoint.py",
             "tests/test_oracle_d3q27.py", "tests/test_oracle_cells_compressible.py",
             "tests/test_oracle_kbc_open.py"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_pins_pass_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
                    "-std=c99", SRC, "-o", lib, "-lm"], check=True)
    env = dict(os.environ, LBM_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    # -s: the sanitizer's report goes to this process's stderr, not to
    # pytest's capture, which an abort would lose
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p",
                          "no:cacheprovider",
                          "-k", "not pressure_driven_channel and not duct_transverse_current",
                          *PIN_FILES], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=900)
    tail = (res.stdout[-3000:] + res.stderr[-3000:])
    assert res.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
