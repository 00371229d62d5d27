"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the library's plan builder (csrc/plan.cpp) and the C oracle, each driven
over random NBB fractals by a small program in tests/sanitize/, compiled
here with g++ / gcc.  Any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]


def _run(cmd_build, exe):
    r = subprocess.run(cmd_build, capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-400:])
    # a library preloaded into every process may come before the sanitizer
    # runtime; tell ASan not to insist on being first
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stdout + r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_plan_builder_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_fuzz")
    out = _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_2110_12952_amd", "csrc"),
                os.path.join(HERE, "plan_fuzz.cpp"), os.path.join(ROOT, "paper_2110_12952_amd", "csrc", "plan.cpp"),
                "-o", exe], exe)
    maps, plans = (int(w) for w in out.split()[1::2])
    assert maps > 300 and plans > 1000


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_fuzz")
    out = _run(["gcc", "-std=c11", *SAN, "-fopenmp", os.path.join(HERE, "oracle_fuzz.c"),
                os.path.join(ROOT, "oracle", "nbb_oracle.c"), "-o", exe], exe)
    assert int(out.split()[1]) > 250
