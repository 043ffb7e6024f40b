"""The C ABI from C: tests/abi_c_host.c is compiled with gcc as strict C99 against
include/rbos.h and linked to the built library, then run on the host (no GPU needed)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2509_14442_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_header_is_c99_and_library_answers_from_c(tmp_path):
    assert os.path.exists(os.path.join(LIBDIR, "librbos.so")), "build the library first"
    exe = str(tmp_path / "abi_c_host")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "abi_c_host.c"), "-L", LIBDIR, "-lrbos", "-Wl,-rpath," + LIBDIR,
                    "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stderr)
    assert out.stdout.strip() == "c abi ok"
