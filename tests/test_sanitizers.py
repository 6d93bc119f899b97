"""Sanitizer runs of the host code, on the CPU.

* The oracle built with gcc's AddressSanitizer and UndefinedBehaviorSanitizer
  (no recovery: the first report aborts) runs under its pins.
* The library built with the same sanitizers on its host side (hipcc, each
  -fsanitize after -Xarch_host; the device code is unchanged) runs under the
  C-ABI tests (validation of problem descriptions before any device work,
  export table) and the linkage-model tests (the host set cover and DSATUR
  colouring against the reference).

Each run is a subprocess with the sanitizer runtime preloaded, so a report
fails the run; leak checking is off (the interpreter's own allocations are
not this code's)."""
import glob
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


def run_pytest(files, env):
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + files
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    return out


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="morea_sanitize_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def test_oracle_under_asan_and_ubsan(workdir):
    gcc_asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    gcc_ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(gcc_asan) or not os.path.exists(gcc_asan):
        pytest.skip("gcc's sanitizer runtime is not installed")
    lib = os.path.join(workdir, "liboracle_sanitized.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", lib, os.path.join(ROOT, "oracle", "morea_oracle.c"),
                           "-lm"])
    env = dict(os.environ, MOREA_ORACLE_LIB=lib, LD_PRELOAD=f"{gcc_asan}:{gcc_ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run_pytest(["tests/test_oracle_pins.py", "tests/test_oracle_sobol.py", "tests/test_oracle_dvf.py",
                "tests/test_oracle_point_guidance.py", "tests/test_oracle_surrogate_inputs.py"], env)


def test_library_host_code_under_asan_and_ubsan(workdir):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt or not os.path.exists(HIPCC):
        pytest.skip("hipcc or its sanitizer runtime is not installed")
    lib = os.path.join(workdir, "libmorea_host_sanitized.so")
    csrc = sorted(glob.glob(os.path.join(ROOT, "paper_2303_04873_amd", "csrc", "*.hip")))
    subprocess.check_call([HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"), "-o", lib] + csrc,
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    env = dict(os.environ, MOREA_LIB=lib, LD_PRELOAD=rt[-1], ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run_pytest(["tests/test_abi.py", "tests/test_oracle_fos.py"], env)
