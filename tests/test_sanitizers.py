"""Host sanitizer runs (CPU only): the C oracle and the library's host-side C
ABI layer built with AddressSanitizer and UndefinedBehaviorSanitizer
(device code is not instrumented), driven by small C programs under
tests/sanitize/ that exercise every oracle routine and every validation path
of the ABI.  A sanitizer report or a wrong return value fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2008_01567_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = "-fsanitize=address,undefined"
ENV_ASAN = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:halt_on_error=1",
            "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, env=None, timeout=600):
    e = dict(os.environ)
    e.update(env or {})
    r = subprocess.run(cmd, capture_output=True, text=True, env=e, timeout=timeout)
    return r.returncode, r.stdout, r.stderr


def _clean(rc, out, err):
    bad = ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:", "FAILED")
    return rc == 0 and not any(b in err for b in bad)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    rc, out, err = _run(["gcc", SAN, "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1",
                         "-std=c11", "-fopenmp", os.path.join(ROOT, "oracle", "oracle.c"),
                         os.path.join(HERE, "oracle_driver.c"), "-o", exe, "-lm"])
    assert rc == 0, err
    rc, out, err = _run([exe], env=dict(ENV_ASAN, OMP_NUM_THREADS="4"), timeout=300)
    print(out, err[-2000:])
    assert _clean(rc, out, err) and "clean" in out


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not available")
def test_c_abi_validation_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "libmsf_asan.so")
    srcs = [os.path.join(CSRC, s) for s in ("capi.hip", "projector.hip", "cg.hip", "cnn.hip", "mace.hip",
                                            "fixture.hip", "exact.hip")]
    # host code instrumented (-Xarch_host before each sanitizer flag), device code built as usual
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), *srcs, "-o", lib]
    rc, out, err = _run(cmd, timeout=900)
    assert rc == 0, err[-3000:]
    exe = str(tmp_path / "abi_asan")
    rc, out, err = _run([CLANG, SAN, "-fno-omit-frame-pointer", "-g", "-O1", "-I", os.path.join(ROOT, "include"),
                         os.path.join(HERE, "abi_driver.c"), "-L", str(tmp_path), "-lmsf_asan",
                         "-Wl,-rpath," + str(tmp_path), "-lm", "-o", exe])
    assert rc == 0, err
    rc, out, err = _run([exe], env=ENV_ASAN, timeout=300)
    print(out, err[-2000:])
    assert _clean(rc, out, err) and "clean" in out
