"""Mapping of the device status word to return codes (host only, no GPU).

A pair whose reverse pair the search did not find would leave a wrong force;
mtp_eval and mtp_status must then fail with MTP_E_STATE instead of returning
success.  The mapping is plain C++ (csrc/status.h), compiled here with g++.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_status_word_maps_to_return_codes(tmp_path):
    exe = tmp_path / "status_code_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_2007_08555_amd", "csrc"),
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "cpp", "status_code_test.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "status mapping ok" in out.stdout
