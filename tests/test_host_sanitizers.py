"""The C ABI's host-side code under AddressSanitizer + UndefinedBehavior-
Sanitizer (CPU only).

api.hip, which holds the library's host logic (parameter validation, layout
and link-word sizes, the storage-scale rule, the velocity-set export and the
argument checks of lbm_init), is compiled with the sanitizers on its host
pass only (-Xarch_host before each -fsanitize flag; the device code is built
as usual) and linked with the library's other objects into a copy of the
package.  The ABI test file then runs against that copy in a fresh process
with clang's sanitizer runtime preloaded: any out-of-bounds access, use
after free or undefined operation in the host code it reaches aborts that
process and fails this test.  Host code behind the GPU allocations of
lbm_init (the collision constants, the active-block list) needs a GPU and is
not reached here.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

from paper_1803_04937_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
            "-g"]


def _runtime():
    hits = sorted(glob.glob(os.path.join(os.path.dirname(os.path.dirname(B.HIPCC)), "llvm", "lib",
                                         "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    return hits[-1] if hits else None


def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    rt = _runtime()
    if rt is None:
        pytest.skip("clang sanitizer runtime not installed")
    others = [os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o") for s in B.SOURCES
              if s != "api.hip"]
    if not all(os.path.exists(o) for o in others):
        pytest.skip("library objects not built (python -m paper_1803_04937_amd.build)")
    api = str(tmp_path / "api_san.o")
    subprocess.run([B.HIPCC, *B.FLAGS, *SANITIZE, "-c", os.path.join(B.CSRC, "api.hip"),
                    "-o", api], check=True, capture_output=True)
    root = tmp_path / "root"
    pkg = root / "paper_1803_04937_amd"
    (root / "tests").mkdir(parents=True)
    pkg.mkdir()
    for f in glob.glob(os.path.join(ROOT, "paper_1803_04937_amd", "*.py")):
        shutil.copy(f, pkg)
    subprocess.run([B.HIPCC, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", *others, api,
                    "-o", str(pkg / "liblbm.so")], check=True, capture_output=True)
    for d in ("oracle", "lbm_inputs", "include"):
        os.symlink(os.path.join(ROOT, d), root / d)
    for f in ("conftest.py", "_helpers.py", "test_abi.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), root / "tests")
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # -s: the sanitizer's report goes to this process's stderr, not to
    # pytest's capture, which an abort would lose
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p",
                          "no:cacheprovider", "tests/test_abi.py"], cwd=str(root), env=env,
                         capture_output=True, text=True, timeout=600)
    tail = res.stdout[-3000:] + res.stderr[-3000:]
    assert res.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
    assert " passed" in res.stdout, tail
