"""CPU sanitizer runs (no GPU):

* the FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, leak
  detection on) and driven through every entry point and variant by tests/san/oracle_driver.c;
* the host half of the C ABI -- argument validation, workspace and scratch sizing, the error
  message, the profiler's host state -- from a build of the library whose host code carries
  both sanitizers (device code unchanged), driven by tests/san/abi_host_driver.c.  Leak
  detection is off there: the HIP runtime's own start-up allocations are not ours."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _run(cmd, env=None, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr[-4000:]}"
    return r.stdout


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_driver")
        _run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all", os.path.join(HERE, "san", "oracle_driver.c"), "-o", exe, "-lm"])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="4")
        out = _run([exe], env=env)
        assert "ok" in out


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_c_abi_host_code_under_address_and_undefined_behaviour_sanitizers():
    from paper_2605_31419_amd import build as B

    clang = "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(clang):
        clang = shutil.which("clang") or pytest.skip("needs clang")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "libtsr_san.so")
        srcs = [os.path.join(B.CSRC, s) for s in B.SOURCES]
        flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g", "-Xarch_host", "-fsanitize=address",
                                                     "-Xarch_host", "-fsanitize=undefined"]
        _run([B.HIPCC, *flags, "-I", B.INCLUDE, "-I", B.CSRC, *srcs, "-o", lib], timeout=600)
        exe = os.path.join(d, "abi_host_driver")
        _run([clang, "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", B.INCLUDE,
              os.path.join(HERE, "san", "abi_host_driver.c"), "-o", exe, f"-L{d}", "-ltsr_san", f"-Wl,-rpath,{d}"])
        out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
        assert "ok" in out
