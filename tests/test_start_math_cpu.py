"""The table-driven segment-start factors of the pair-G passes (exponential by
Tang's table method, e^{-2 pi i f} by a 64-step table and Taylor series; see
csrc/kernel_common.h), compiled for the host from the same source the kernels
use and checked against long double references over the argument ranges of the
kernels: about 1 ulp for the exponential, 1.2e-16 absolute for cos / sin."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2509_16460_amd", "csrc")


def test_start_factors_accuracy(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "start_math_check")
    subprocess.check_call([gxx, "-O2", "-std=c++17", "-D__host__=", "-D__device__=", "-D__forceinline__=inline", "-I", CSRC,
                           os.path.join(HERE, "start_math_check.cpp"), "-o", exe])
    out = subprocess.check_output([exe], text=True).split()
    exp_ulp, cis_abs = float(out[1]), float(out[3])
    print(f"exp_tab max error {exp_ulp:.3f} ulp, cis_neg max error {cis_abs:.2e}")
    assert exp_ulp <= 1.5
    assert cis_abs <= 2.5e-16
