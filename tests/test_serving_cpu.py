"""Host-only checks of the serving scheduler core (paper_2507_16022_amd/csrc/serving.h):
first-fit pool map, FIFO admission by memory, slot limit, drain on destruction."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2507_16022_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scheduler_core(tmp_path):
    exe = str(tmp_path / "serving_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-pthread", "-I", CSRC,
                    os.path.join(HERE, "native", "serving_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    assert "serving_check OK" in out.stdout
