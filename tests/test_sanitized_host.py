"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle's C source and the library's background cosmology, each
driven through every entry point by a small program in tests/sanitize/."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_and_run(cmd, exe):
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("no sanitizer runtime: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout, run.stderr[-2000:])
    assert run.returncode == 0, run.stderr[-2000:]
    assert "ERROR: AddressSanitizer" not in run.stderr
    assert "runtime error" not in run.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _build_and_run(["gcc", "-std=c11", "-fopenmp"] + SAN +
                   [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                    "-o", exe, "-lm"], exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_background_under_sanitizers(tmp_path):
    exe = str(tmp_path / "cosmo_driver")
    csrc = os.path.join(ROOT, "paper_1811_05903_amd", "csrc")
    _build_and_run(["g++", "-std=c++17"] + SAN +
                   ["-I" + csrc, os.path.join(ROOT, "tests", "sanitize", "cosmo_driver.cpp"),
                    os.path.join(csrc, "steps_cosmo.cpp"), "-o", exe], exe)
