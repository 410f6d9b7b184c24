"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

- libhj: every source rebuilt with the sanitizers on its host code only (the
  gfx950 device code is built as usual), loaded in place of the in-tree
  library (HJ_LIB_PATH) with the compiler's ASan runtime preloaded, runs the
  library's CPU tests: the exported boundary, argument errors of every entry
  point, the binding's checks and the injected allocation failure.
- oracle: built with the same sanitizers by gcc, runs the oracle's pins.

A sanitizer report fails the run (halt_on_error); leak checking is off (the
Python interpreter itself holds memory to the end).
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_11542_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run_tests(env_extra, files, threads="2"):
    env = dict(os.environ, OMP_NUM_THREADS=threads, **SAN_ENV, **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] +
                       [os.path.join(ROOT, "tests", f) for f in files],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_libhj_host_code_under_asan_ubsan(tmp_path):
    runtime = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not runtime or not os.path.exists(HIPCC):
        pytest.skip("no clang ASan runtime or hipcc")
    sources = sorted(glob.glob(os.path.join(CSRC, "*.cpp")) + glob.glob(os.path.join(CSRC, "*.hip")))
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-I" + os.path.join(ROOT, "include")] + san

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([HIPCC] + flags + ["-c", src, "-o", obj], capture_output=True,
                           text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, sources))
    lib = str(tmp_path / "libhj_san.so")
    r = subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950"] + san[:4] +
                       ["-o", lib] + objs, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = _run_tests({"HJ_LIB_PATH": lib, "LD_PRELOAD": runtime[0]},
                     ["test_abi.py", "test_binding_checks.py"])
    assert " passed" in out


def test_oracle_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no gcc ASan runtime")
    lib = str(tmp_path / "libhj_oracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-std=c99", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-o", lib, os.path.join(ROOT, "oracle", "hj_oracle.c"), "-lm"], check=True)
    out = _run_tests({"HJ_ORACLE_LIB": lib, "LD_PRELOAD": asan},
                     ["test_oracle_pins.py", "test_oracle_storage_model.py",
                      "test_oracle_shapes.py", "test_oracle_dissipation.py",
                      "test_oracle_rockets_tubes.py"])
    assert " passed" in out
