"""The C ABI from plain C: `include/rtsun.h` compiles as pedantic C99 and a C
program linked against librtsun.so gets the constants, defaults and every
host-side argument check through it (CPU only: no call reaches a device)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_header_is_c99_and_host_checks_hold_from_c(tmp_path):
    from paper_2606_02413_amd import rtsun
    if not os.path.exists(rtsun.LIB_PATH):
        from paper_2606_02413_amd import build
        build.build()
    libdir = os.path.dirname(rtsun.LIB_PATH)
    exe = str(tmp_path / "abi_host_check")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "abi_host_check.c"), "-o", exe, "-L", libdir, "-lrtsun", "-lm",
           f"-Wl,-rpath,{libdir}"]
    subprocess.run(cmd, check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
