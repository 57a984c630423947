"""Register DFTs of the HIP FFT engine, built for the host and checked against a direct
FP64 DFT (forward and inverse, with and without runtime twiddles folded into the
butterflies).  Needs g++ and the ROCm headers; no GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1112_1805_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_register_dfts_on_host(tmp_path):
    exe = tmp_path / "host_fft_check"
    # no FMA contraction beyond what the source writes: the explicit fmaf calls are the
    # engine's rounding steps
    cmd = ["g++", "-std=c++17", "-O1", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + CSRC, os.path.join(HERE, "host_fft_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(res.stdout)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("OK")
