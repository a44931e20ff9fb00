"""The CPU code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle (plain C, gcc) and the CPU harnesses of the device arithmetic and
the adjoint (tests/host, host code built by hipcc) are rebuilt with both
sanitizers, errors fatal, and a reduced set of their pin tests runs against
the instrumented builds in a child process that preloads the matching
sanitizer runtime.  A heap overflow, a use after free, a signed overflow, a
misaligned or out-of-bounds access ends that process with an error.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
# the slow convergence scans are left out; every other pin runs
SLOW = "not diagonal_wave_second_order and not positivity_on_workload_shapes and not sod_converges"


def _symbols(lib):
    r = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True)
    return r.stdout


def _run(env, files, k=None):
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *files]
    if k:
        cmd += ["-k", k]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                    "-o", lib, os.path.join(ROOT, "oracle", "cshoracle.c"),
                    os.path.join(ROOT, "oracle", "cshoracle3.c"), "-lm"], check=True)
    syms = _symbols(lib)
    assert "__asan_report" in syms and "__ubsan_handle" in syms
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    env = dict(os.environ, CSH_ORACLE_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0",
               OMP_NUM_THREADS="2")
    files = [os.path.join(TESTS, f) for f in ("test_oracle_branch_pins.py", "test_oracle_pins.py",
                                              "test_oracle_kt_pins.py", "test_oracle_hllc_pins.py",
                                              "test_oracle_fourier_pins.py", "test_oracle3_pins.py")]
    _run(env, files, SLOW)


def test_host_harnesses_under_asan_ubsan():
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt:
        pytest.skip("clang's ASan runtime not found")
    env = dict(os.environ, CSH_HOST_SANITIZE="1")
    sys.path.insert(0, os.path.join(TESTS, "host"))
    import build_host
    build_host.SANITIZE = True
    try:
        libs = [build_host.build(), build_host.build_device()]
    finally:
        build_host.SANITIZE = False
    for lib in libs:
        syms = _symbols(lib)
        assert "__asan_report" in syms and "__ubsan_handle" in syms, lib
    env.update(LD_PRELOAD=rt[0], ASAN_OPTIONS="detect_leaks=0")
    _run(env, [os.path.join(TESTS, "test_adjoint_host.py"), os.path.join(TESTS, "test_device_arith_host.py")])
