"""The batched solve forms its scalings u = (a/s)^fi with the library's own FP64
log and exp (paper_2412_11079_amd/csrc/scalemath.h: the atanh series for
log, Cody-Waite reduction and the Taylor series for exp).  The same header
is compiled here for the host with g++ and checked against long-double
libm over the normal and subnormal range: log within 4 ulp of max(|log x|,
1), exp within 4 ulp, the scaling power within 8 units of its conditioning,
and the special totals (0, inf, NaN) as the plain formula gives them."""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2412_11079_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_scaling_log_exp_against_long_double(tmp_path):
    exe = str(tmp_path / "scalemath_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I" + CSRC, os.path.join(HERE, "cpp", "scalemath_check.cpp"),
                    "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    vals = dict(re.findall(r"(\w+)=([0-9.]+)", out))
    assert float(vals["log_ulps"]) <= 4.0, out
    assert float(vals["exp_ulps"]) <= 4.0, out
    assert float(vals["pow_units"]) <= 8.0, out
    assert vals["specials"] == "1", out
