"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the oracle and the
CPU-parallel baseline, compiled with tests/sanitize_oracle.cpp (random read sets for every
k, the extension and query entry points, edge cases and bad arguments; every parallel
result compared with the oracle's).  Any sanitizer report aborts the driver."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_and_parallel_baseline_clean_under_asan_ubsan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no C++ compiler")
    exe = tmp_path / "san_oracle"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", str(exe),
           os.path.join(HERE, "sanitize_oracle.cpp"), os.path.join(ROOT, "oracle", "kc_oracle.cpp"),
           os.path.join(ROOT, "oracle", "kc_cpu_parallel.cpp")]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="8")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "0 mismatches" in out
