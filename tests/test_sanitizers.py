"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the CPU (no GPU needed):

* the oracle (plain C) built with both sanitizers runs every entry point on small seeded inputs
  with odd sizes, border and out-of-image points, every tracker form, the gradients, the global
  fit and the dense interpolation (tests/sanitize/oracle_checks.c);
* the HIP library's host code built with both sanitizers (device code unchanged) runs the
  argument validation of every C-ABI entry point, each call stopping before any device work
  (tests/sanitize/abi_checks.c).

A pass is exit status 0 with no sanitizer report."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ROCM = "/opt/rocm"
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
HIPCC = os.path.join(ROCM, "bin", "hipcc")


def _run(cmd, env=None, timeout=300):
    p = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return p.returncode, p.stdout + p.stderr


def test_oracle_under_asan_and_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_checks")
    rc, out = _run(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fopenmp", os.path.join(HERE, "oracle_checks.c"), os.path.join(ROOT, "oracle", "degraf_oracle.c"),
                    os.path.join(ROOT, "oracle", "epic_oracle.c"), "-lm", "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    rc, out = _run([exe], env=env)
    assert rc == 0 and "passed" in out and "Sanitizer" not in out, out


def test_host_validation_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not available")
    srcs = sorted(os.path.join(ROOT, "paper_1901_09971_amd", "csrc", f)
                  for f in os.listdir(os.path.join(ROOT, "paper_1901_09971_amd", "csrc")) if f.endswith(".hip"))
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # sanitizers on the host code only
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all",
             "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1901_09971_amd", "csrc")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src)[:-4] + ".o"))
        rc, out = _run([HIPCC, *flags, "-c", src, "-o", obj], timeout=600)
        assert rc == 0, out
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libdgf_asan.so")
    rc, out = _run([CLANG + "++", "-shared", "-fsanitize=address,undefined", *objs, "-L" + os.path.join(ROCM, "lib"),
                    "-lamdhip64", "-o", lib])
    assert rc == 0, out
    exe = str(tmp_path / "abi_checks")
    rc, out = _run([CLANG, "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "abi_checks.c"), lib,
                    "-Wl,-rpath," + str(tmp_path), "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
                    "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lm", "-o", exe])
    assert rc == 0, out
    # the HIP runtime keeps its allocations to the end of the process: leaks are not checked here
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([exe], env=env)
    assert rc == 0 and "passed" in out and "Sanitizer" not in out, out
