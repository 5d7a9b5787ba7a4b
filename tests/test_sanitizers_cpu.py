"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer.

libobk is built with the sanitizers on its host code (-Xarch_host, so the
gfx950 code is unchanged) and the oracle with the same compiler and
sanitizers; the CPU tests that run host code (the oracle's pins, the banded
engine's layout and emulation, the plan validator, the ABI's host entry
points) then run in a child process with the sanitizer runtime preloaded,
and any report ends it.  A control build with a planted heap overflow shows
that a report does end the child.  No device is used."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitized")
CLANG = "/opt/rocm/llvm/bin/clang"
RT_DIR = "/opt/rocm/llvm/lib/clang"
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-shared-libsan",
       "-fno-omit-frame-pointer"]


def _asan_runtime():
    for ver in sorted(os.listdir(RT_DIR), reverse=True):
        p = os.path.join(RT_DIR, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


def _env():
    env = dict(os.environ)
    env.update(LD_PRELOAD=_asan_runtime(), LD_LIBRARY_PATH="/opt/rocm/llvm/lib",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="2")
    return env


@pytest.fixture(scope="module")
def sanitized():
    if not (os.path.exists(CLANG) and _asan_runtime()):
        pytest.skip("the ROCm LLVM toolchain with its sanitizer runtime is not installed")
    os.makedirs(OUT, exist_ok=True)
    oracle_lib = os.path.join(OUT, "liboracle_san.so")
    subprocess.run([CLANG, "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", *SAN,
                    "-shared", "-fPIC", "-o", oracle_lib, os.path.join(ROOT, "oracle", "obk_oracle.c"), "-lm"],
                   check=True)
    spec = importlib.util.spec_from_file_location("obk_build_san", os.path.join(ROOT, "paper_2401_00672_amd",
                                                                                "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    b.OUT_DIR = os.path.join(OUT, "obj")
    b.COMMON = b.COMMON + [f for s in SAN for f in ("-Xarch_host", s)]
    os.makedirs(b.OUT_DIR, exist_ok=True)
    objs = [b._compile(src) for src in b.SOURCES]
    obk_lib = os.path.join(OUT, "libobk_san.so")
    subprocess.run([b.HIPCC, f"--offload-arch={b.ARCH}", "-shared", "-fPIC", *SAN[:3], "-shared-libsan", "-o",
                    obk_lib, *objs], check=True)
    return obk_lib, oracle_lib


@pytest.mark.timeout(1200)
def test_host_code_clean_under_sanitizers(sanitized):
    obk_lib, oracle_lib = sanitized
    env = _env()
    env.update(OBK_LIB=obk_lib, OBK_ORACLE_LIB=oracle_lib)
    tests = ["tests/test_oracle_pins.py", "tests/test_banded_cpu.py", "tests/test_validate_cpu.py",
             "tests/test_abi_cpu.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1100)
    out = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out


def test_a_planted_overflow_is_reported(tmp_path):
    """Control: one byte read past a heap block, in a library built the same
    way, ends the child with an AddressSanitizer report."""
    if not (os.path.exists(CLANG) and _asan_runtime()):
        pytest.skip("the ROCm LLVM toolchain with its sanitizer runtime is not installed")
    src = tmp_path / "overflow.c"
    src.write_text("#include <stdlib.h>\nint over(int n){char*p=malloc(n);int v=p[n];free(p);return v;}\n")
    lib = tmp_path / "liboverflow.so"
    subprocess.run([CLANG, "-O0", *SAN, "-shared", "-fPIC", "-o", str(lib), str(src)], check=True)
    code = f"import ctypes; ctypes.CDLL({str(lib)!r}).over(16)"
    r = subprocess.run([sys.executable, "-c", code], env=_env(), capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
