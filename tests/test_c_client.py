"""The C ABI from plain C: include/ss.h compiles as C99 and a C client
links against libss.so (CPU); the client solves a closed-form case on the
GPU (gpu marker)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "abi_client.c")
LIBDIR = os.path.join(ROOT, "paper_1504_06768_amd")


def _build(tmp_path):
    exe = str(tmp_path / "abi_client")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), SRC,
           "-L", LIBDIR, "-lss", f"-Wl,-rpath,{LIBDIR}", "-lm", "-o", exe]
    if not os.path.exists(os.path.join(LIBDIR, "libss.so")):
        pytest.skip("libss.so not built")
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def test_header_is_c99_and_client_links(tmp_path):
    assert os.path.exists(_build(tmp_path))


@pytest.mark.gpu
def test_c_client_solves_the_coherent_state(tmp_path):
    exe = _build(tmp_path)
    r = subprocess.run([exe, "40"], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
