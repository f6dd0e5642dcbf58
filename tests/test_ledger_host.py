"""The process-wide ledger of split-unit members (device-wide co-residency
bound shared by all contexts), checked on the host: the ledger header is
compiled with g++ into a small driver that exercises its accounting, also
under concurrent reservations from many threads."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1906_11195_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "native", "ledger_check.cpp")


def test_split_ledger_accounting(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("needs g++")
    exe = str(tmp_path / "ledger_check")
    subprocess.check_call([gxx, "-O1", "-std=c++17", "-pthread", "-I" + CSRC, SRC, "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ledger ok" in out.stdout
