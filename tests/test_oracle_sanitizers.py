"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/oracle_sanitize.c calls every entry point of oracle/wilson_oracle.c on
small lattices (ragged extents, 1-4 columns) with two OpenMP threads; the
program stops at the first sanitizer report (-fno-sanitize-recover=all) and
checks <phi, D psi> = <D^H phi, psi>, A = D^H D and the
site-sampled forms, so a report or a failed check fails the test.  Built
with ROCm's clang: its AddressSanitizer sees the complex-double stores of
the stencil (an output buffer one element short is reported), which gcc 11's
misses.  One allocation of the OpenMP runtime itself, which it never frees,
is suppressed from the leak report."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CLANG = "/opt/rocm/llvm/bin/clang"
OMP_LIB = "/opt/rocm/llvm/lib"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not available")
def test_oracle_c_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = [CLANG, "-std=c11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "oracle_sanitize.c"), os.path.join(ROOT, "oracle", "wilson_oracle.c"),
           "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:___kmp_allocate\n")
    env = dict(os.environ, OMP_NUM_THREADS="2",
               LD_LIBRARY_PATH=OMP_LIB + os.pathsep + os.environ.get("LD_LIBRARY_PATH", ""),
               ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               LSAN_OPTIONS=f"suppressions={supp}",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.stdout.count("0 failed checks") == 4
