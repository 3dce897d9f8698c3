"""Arithmetic identities the kernels rely on, checked exhaustively on the
CPU (IEEE binary32 with fused multiply-add, as on the GPU)."""
import os
import subprocess

import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.slow
def test_division_free_divide_by_three_is_correctly_rounded(tmp_path):
    exe = str(tmp_path / "div3")
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", os.path.join(GOLD, "div3_check.c"),
                    "-lm", "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.strip()
    assert out == "0"
