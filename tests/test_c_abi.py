"""The C ABI from C: tests/c_abi_check.c is compiled as strict C99 against
include/*.h with gcc, linked with liblbmhd.so and run (host-only calls)."""

import os
import shutil
import subprocess

import pytest

from paper_1705_09807_amd import native as N

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_headers_compile_as_c_and_host_calls_behave(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    if not os.path.exists(N.LIB_PATH):
        pytest.fail("liblbmhd.so is not built; run __graft_entry__.build() first")
    exe = tmp_path / "c_abi_check"
    libdir = os.path.dirname(N.LIB_PATH)
    cmd = [gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "c_abi_check.c"), "-o", str(exe), "-L", libdir, "-llbmhd", f"-Wl,-rpath,{libdir}"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "c abi ok" in out.stdout
