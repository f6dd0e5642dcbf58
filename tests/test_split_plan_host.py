"""The planner that splits large VB units over several workgroups, checked
on the host: the planner header is compiled with g++ into a small driver
that checks the members it gives equal and unequal graphs, resident units,
forced plans and tight budgets."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1906_11195_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "native", "split_plan_check.cpp")


def test_split_plan_members(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("needs g++")
    exe = str(tmp_path / "split_plan_check")
    subprocess.check_call([gxx, "-O1", "-std=c++17", "-I" + CSRC, SRC, "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "split plan ok" in out.stdout
