"""The FP64 x^p of the general-p kernel kind (pow64.hpp: 2^(p log2 x) by an
atanh series for log2 and a Taylor series for 2^f), built for the host with
g++ and checked against 40-digit decimal powers: relative error within the
header's stated bound (|p log2 x| + 8) * 2^-52, exact at x = 0 and 1."""
import ctypes
import os
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_07183_amd", "csrc")
DRIVER = r'''
#include "pow64.hpp"
extern "C" void pow_many(const double *x, const double *p, double *out, long n) {
    for (long i = 0; i < n; ++i) out[i] = pcf::pow_series(x[i], p[i]);
}
'''


@pytest.fixture(scope="module")
def pow_many(tmp_path_factory):
    d = tmp_path_factory.mktemp("pow64")
    src, lib = d / "drv.cpp", d / "libdrv.so"
    src.write_text(DRIVER)
    subprocess.run(["g++", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-I", CSRC,
                    str(src), "-o", str(lib)], check=True)
    f = ctypes.CDLL(str(lib)).pow_many
    D = ctypes.POINTER(ctypes.c_double)

    def run(x, p):
        x, p = np.ascontiguousarray(x, float), np.ascontiguousarray(p, float)
        out = np.empty_like(x)
        f(x.ctypes.data_as(D), p.ctypes.data_as(D), out.ctypes.data_as(D), ctypes.c_long(len(x)))
        return out
    return run


def test_against_decimal(pow_many):
    getcontext().prec = 40
    rng = np.random.default_rng(3)
    x = np.exp(rng.uniform(np.log(1e-8), np.log(1e8), 3000))
    x[:40] = rng.uniform(0.6, 1.6, 40)  # around the reduction boundary sqrt(2)
    x[40:44] = [np.sqrt(0.5), np.sqrt(2.0), 0.5, 2.0]
    p = rng.uniform(1.0, 10.0, 3000)
    p[:500] = 2.7
    got = pow_many(x, p)
    for xi, pi, gi in zip(x, p, got):
        ref = Decimal(float(xi)) ** Decimal(float(pi))
        if not Decimal("1e-300") < ref < Decimal("1e300"):
            continue
        bound = (abs(pi * np.log2(xi)) + 8) * 2.0 ** -52
        assert float(abs((Decimal(float(gi)) - ref) / ref)) <= bound, (xi, pi, gi)


def test_special_values(pow_many):
    assert pow_many([0.0, 1.0, 1.0], [2.7, 2.7, 9.3]).tolist() == [0.0, 1.0, 1.0]
    out = pow_many([1e-200, 1e200], [3.3, 3.3])
    assert out[0] == 0.0 and out[1] == np.inf
