"""The FP64 oracle and the library's host-side parameter checks built with the address and
undefined-behaviour sanitizers (host code only, gcc / g++) and run on small seeded
scenarios and on every kind of invalid parameter: any out-of-bounds access, leak, overflow
or undefined operation aborts the driver (no recovery), which fails the test."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]


def _build_and_run(tmp_path, compiler, std, sources, includes, extra=()):
    exe = str(tmp_path / "driver")
    cmd = [compiler, std, *SAN, *extra, *(f"-I{i}" for i in includes), *sources, "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stderr[-4000:]
    return run.stdout


def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc", "-std=c11",
                         [os.path.join(ROOT, "oracle", "cuesim_oracle.c"),
                          os.path.join(HERE, "oracle_driver.c")],
                         [os.path.join(ROOT, "oracle")], extra=["-fopenmp"])
    assert "ok" in out


def test_parameter_checks_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1405_3331_amd", "csrc")
    out = _build_and_run(tmp_path, "g++", "-std=c++17",
                         [os.path.join(csrc, "validate.cpp"),
                          os.path.join(HERE, "validate_driver.cpp")],
                         [os.path.join(ROOT, "include"), csrc])
    assert "ok" in out
