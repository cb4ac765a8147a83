"""CPU runs of host code under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU
oracle (plain C) through every entry point, the library's host-side setup arithmetic
(parameter resolution, primes, roots, tables, twiddles) and its tuning-file module.  The serving runtime's host
bookkeeping has its own sanitized test (test_runtime_cpu.py)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(exe, *args):
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip() == "OK"


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-std=c11", *SAN, "-ffp-contract=off", "-D_GNU_SOURCE", "-fopenmp", "-o", exe,
                    os.path.join(HERE, "native", "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "ckks_oracle.c"),
                    "-lm"], check=True, capture_output=True)
    _run(exe)


def test_library_host_math_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_math_san")
    subprocess.run(["g++", "-std=c++17", *SAN, "-ffp-contract=off", "-o", exe,
                    os.path.join(HERE, "native", "host_math_sanitize_driver.cpp"),
                    os.path.join(ROOT, "paper_2409_03568_amd", "csrc", "host_math.cpp")], check=True, capture_output=True)
    _run(exe)


def test_tune_file_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tune_file_san")
    subprocess.run(["g++", "-std=c++17", *SAN, "-o", exe, os.path.join(HERE, "native", "tune_file_test.cpp"),
                    os.path.join(ROOT, "paper_2409_03568_amd", "csrc", "tune_file.cpp")], check=True,
                   capture_output=True)
    scratch = tmp_path / "scratch"
    scratch.mkdir()
    _run(exe, str(scratch))
