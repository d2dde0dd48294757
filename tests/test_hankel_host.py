"""The device Hankel evaluator (csrc/hbi_hankel.h) compiled for the host
with g++ and checked against SciPy's Bessel functions over (0, 3000], each
branch (series, Miller recurrence, asymptotic expansion) and its edges."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import special

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2210_02698_amd", "csrc")

SRC = r'''
#define HBI_HD
#include "hbi_hankel.h"
extern "C" void eval(const double *x, double *out, int n) {
  for (int i = 0; i < n; ++i) {
    const hbi::Hankel01 h = hbi::hankel01(x[i]);
    out[4 * i] = h.j0; out[4 * i + 1] = h.y0; out[4 * i + 2] = h.j1; out[4 * i + 3] = h.y1;
  }
}
'''


@pytest.fixture(scope="module")
def hankel_lib():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "h.cpp")
    so = os.path.join(d, "h.so")
    open(src, "w").write(SRC)
    subprocess.check_call(["g++", "-O2", "-shared", "-fPIC", "-I", CSRC, src, "-o", so])
    lib = ctypes.CDLL(so)
    lib.eval.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    return lib


def evaluate(lib, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty((x.size, 4))
    lib.eval(x.ctypes.data, out.ctypes.data, x.size)
    return out


def test_hankel_matches_scipy(hankel_lib):
    rng = np.random.default_rng(3)
    x = np.concatenate([
        np.geomspace(1e-3, 3.0, 400), np.linspace(3.0, 20.0, 2000),
        np.geomspace(20.0, 3000.0, 2000), rng.uniform(0.01, 50.0, 2000),
        # both sides of the branch points
        np.array([3.0 - 1e-12, 3.0, 3.0 + 1e-12, 20.0 - 1e-12, 20.0, 20.0 + 1e-12])])
    got = evaluate(hankel_lib, x)
    for k, (nu, kind) in enumerate([(0, "j"), (0, "y"), (1, "j"), (1, "y")]):
        ref = special.jv(nu, x) if kind == "j" else special.yv(nu, x)
        # error relative to the modulus of the Hankel function of that order
        mod = np.hypot(special.jv(nu, x), special.yv(nu, x))
        err = np.abs(got[:, k] - ref) / mod
        assert err.max() < 5e-15, (nu, kind, float(err.max()), float(x[np.argmax(err)]))
