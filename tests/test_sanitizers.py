"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle's C library and the library's host set-up code, each
built with gcc/g++ and -fsanitize=address,undefined into a driver program
that calls every routine on small grids (tests/sanitize/).  A sanitizer
report aborts the driver, so the test passes only on a clean run."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _build_and_run(cmd, exe, expect):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV)
    assert r.returncode == 0 and expect in r.stdout, r.stdout + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-std=c99", "-fopenmp"] + SAN + ["-I", os.path.join(ROOT, "oracle"),
                                                    os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                                                    os.path.join(ROOT, "oracle", "numa_oracle.c"), "-lm", "-o", exe]
    _build_and_run(cmd, exe, "oracle driver ok")


def test_host_setup_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_ops_driver")
    csrc = os.path.join(ROOT, "paper_1702_04316_amd", "csrc")
    cmd = ["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", csrc] + SAN + [
        os.path.join(ROOT, "tests", "sanitize", "host_ops_driver.cpp"), os.path.join(csrc, "setup.cpp"), "-o", exe]
    _build_and_run(cmd, exe, "host ops driver ok")
