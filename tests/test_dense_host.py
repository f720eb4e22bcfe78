"""Host dense kernels of the coarse factorisation (csrc/dense_host.cpp).

The multifrontal LU of K_g is factored once per model on the host; its dense
kernels (blocked elimination, multiply-accumulate, triangular inverses, the
thread team) must give every entry the same bits as the textbook loops, so
that the factors do not depend on blocking or thread count.  The check
program (tests/dense_host_check.cpp) is built from the library's own source
with the library's host flags and compares bit for bit, plus the inverse
residual and the zero-pivot report.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2501_06748_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_dense_kernels_match_textbook_loops(tmp_path):
    from paper_2501_06748_amd.build import HOST_FLAGS

    exe = tmp_path / "dense_host_check"
    cmd = ["g++", *HOST_FLAGS, "-I", CSRC, os.path.join(HERE, "dense_host_check.cpp"),
           os.path.join(CSRC, "dense_host.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
