"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code, gcc), driving
every one of its entry points once on a small scene with every loss term, open and closed items, an
empty item and an item partly off its canvas (oracle/sanitize_check.c).  Any out-of-bounds access,
use after free, leak or undefined operation aborts the program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    src = os.path.join(ROOT, "oracle", "sanitize_check.c")
    cmd = ["gcc", "-std=c99", "-g", "-O1", "-Wall", "-Wno-unknown-pragmas", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"), src, "-lm",
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert res.returncode == 0 and res.stdout.strip() == "ok", res.stdout + res.stderr
