"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

oracle/sanitize_check.cpp calls every entry point of the oracle once on small
inputs; built with -fsanitize=address,undefined (no recovery), any invalid
memory access, leak or undefined operation ends the program with an error.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-pthread", os.path.join(ROOT, "oracle", "sanitize_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, cwd=os.path.join(ROOT, "oracle"))
    # (verify_asan_link_order=0: the environment may preload a library of its own)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip().endswith("ok"), r.stdout
