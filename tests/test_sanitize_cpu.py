"""Host-side memory and undefined-behaviour checks, on the CPU.

The float64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc) runs its
pin tests, and libials with the same sanitizers on its host side only (device code is built
as usual) runs the C-ABI tests, which exercise the argument validation of every entry point
without a GPU.  Each runs in a child process with the sanitizer runtime preloaded; any
sanitizer report fails the test (UBSan stops at the first error, leak detection is off because
the Python interpreter itself is not instrumented)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    if not (os.path.isabs(p) and os.path.exists(p)):
        pytest.skip("no AddressSanitizer runtime for gcc")
    return p


def _clang_runtime():
    # the runtime of the compiler hipcc drives (its shared ASan runtime carries the UBSan handlers)
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        pytest.skip("no AddressSanitizer runtime for the ROCm compiler")
    return hits[-1]


def _run(tests, env_extra, runtime):
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4", **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    lib = tmp_path / "libials_oracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", str(lib),
                    os.path.join(ROOT, "oracle", "ials_oracle.c"), "-lm"], check=True)
    out = _run(["tests/test_oracle_pins.py"], {"IALS_ORACLE_LIB": str(lib)}, _gcc_runtime())
    assert " passed" in out


def test_abi_validation_under_host_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2110_14044_amd import build as hip_build
    lib = str(tmp_path / "libials_san.so")
    hip_build.build(out=lib, build_dir=str(tmp_path / "obj"),
                    host_flags=("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
                                "-fno-omit-frame-pointer"))
    out = _run(["tests/test_abi_cpu.py"], {"IALS_LIB": lib}, _clang_runtime())
    assert " passed" in out
