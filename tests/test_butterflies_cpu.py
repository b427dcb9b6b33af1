"""The register butterflies of the tile kernel (radices 2-16, including the
composites built by one eq. ct step with compile-time twiddles, and the primes
11, 13, 17, 19 and 23), compiled for the host with g++ and checked against the DFT
definition."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2602_23525_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_every_radix_matches_the_definition(tmp_path):
    exe = tmp_path / "butterfly_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", os.path.join(HERE, "host_stub"), "-I", CSRC,
                    os.path.join(HERE, "butterfly_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout
    assert out.stdout.count("radix") == 18
