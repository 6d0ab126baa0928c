"""Accuracy of the FP64 exponential that sets the adapted step sizes and
accept statistics inside the fused logistic kernel (csrc/exp_f64.hpp), compiled
for the host with the kernel's own source and compared against e^x from
Python's decimal module at 50 significant digits (correctly rounded, so an
independent reference, not libm).

Bound: at most 1 ulp of the correctly rounded result over [-745, 709.78]
(measured maximum 0.82 ulp), the subnormal range included; 0 below
-745.2 (where e^x < 2^-1075 rounds to 0), +inf above 709.8, NaN propagated.
"""
import math
import os
import shutil
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2002_01184_amd", "csrc")


@pytest.fixture(scope="module")
def exp_lds(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include/hip"):
        pytest.skip("g++ or HIP headers unavailable")
    exe = str(tmp_path_factory.mktemp("exp") / "exp_f64_check")
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-I" + CSRC, os.path.join(HERE, "exp_f64_check.cpp"),
                           "-o", exe])

    def run(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = subprocess.run([exe], input=x.tobytes(), capture_output=True, check=True).stdout
        return np.frombuffer(out, dtype=np.float64)
    return run


def _ulp_error(x, y):
    getcontext().prec = 50
    errs = np.empty(len(x))
    for i, (xi, yi) in enumerate(zip(x, y)):
        exact = Decimal(float(xi)).exp()
        ref = float(exact)                      # correctly rounded
        ulp = math.ulp(ref) if ref > 0 else math.ulp(0.0)
        errs[i] = float(abs(Decimal(float(yi)) - exact) / Decimal(ulp))
    return errs


def test_exp_lds_within_one_ulp(exp_lds):
    rng = np.random.default_rng(5)
    ln2 = math.log(2.0)
    x = np.concatenate([
        np.linspace(-745.0, 709.78, 6001),
        rng.uniform(-745.0, 709.78, 4000),
        rng.uniform(-40.0, 0.0, 4000),            # the accept statistics and log step sizes live here
        (np.arange(-1074, 1024) + 0.5) * ln2,     # reduction boundaries, |r| = ln2 / 2
        np.arange(-1074, 1024) * ln2,             # r close to 0
        rng.uniform(-1e-6, 1e-6, 200), [0.0, -0.0, 5e-324, -5e-324],
        rng.uniform(-745.0, -708.4, 500),         # subnormal results
    ])
    x = x[(x >= -745.0) & (x <= 709.78)]
    y = exp_lds(x)
    err = _ulp_error(x, y)
    assert np.all(np.isfinite(y))
    assert err.max() <= 1.0, (x[np.argmax(err)], err.max())


def test_exp_lds_edges(exp_lds):
    x = np.array([-745.3, -800.0, -np.inf, 709.9, 1e4, np.inf, np.nan, 0.0])
    y = exp_lds(x)
    assert np.all(y[:3] == 0.0)
    assert np.all(np.isposinf(y[3:6]))
    assert np.isnan(y[6])
    assert y[7] == 1.0
