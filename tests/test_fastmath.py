"""CPU check of the kernels' sine/cosine (Cody-Waite reduction + Taylor
series) against numpy on the arguments the quadratures meet (|k r| <= 1e3)."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2006_02545_amd", "csrc", "check", "fastmath_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_sincos_against_numpy():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-4, 4, 20000), rng.uniform(-1e3, 1e3, 20000),
                        np.arange(-64, 65) * np.pi / 4, [0.0, 1e-300, -1e-20, 5e5, 2e6]])
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "fm")
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", exe, SRC])
        out = subprocess.run([exe], input="\n".join(repr(float(v)) for v in x), text=True,
                             capture_output=True, check=True).stdout
    sc = np.array([[float(t) for t in line.split()] for line in out.strip().splitlines()])
    err_s = np.abs(sc[:, 0] - np.sin(x))
    err_c = np.abs(sc[:, 1] - np.cos(x))
    # absolute error of a few ulp of 1, plus the reduction error ~ |x| 2^-100
    bound = 4.5e-16 + 1e-30 * np.abs(x)
    assert np.all(err_s <= bound), (x[np.argmax(err_s - bound)], err_s.max())
    assert np.all(err_c <= bound), (x[np.argmax(err_c - bound)], err_c.max())
