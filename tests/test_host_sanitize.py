"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
checkpoint header parser of the library (paper_1311_4627_amd/csrc/hsd_ckpt.h),
built with g++ into a standalone harness and fed truncated, corrupted and
edited checkpoint images (tests/sanitize/ckpt_fuzz.cpp).  No GPU code is
built with a sanitizer."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_checkpoint_parser_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    exe = str(tmp_path / "ckpt_fuzz")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "paper_1311_4627_amd", "csrc"),
           os.path.join(ROOT, "tests", "sanitize", "ckpt_fuzz.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("the sanitizer runtimes are not installed: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(run.stdout[-500:])
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-2000:]
    assert "ok: 0 failures" in run.stdout
