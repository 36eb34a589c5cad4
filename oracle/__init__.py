"""CPU oracle for PCF pairwise integrated-combination matrices.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, single-threaded FP64
reference written from the paper's definitions (Section 2, Section 2.2
"Functionals", Section 3 Eq. "simpleint", Section 3.1 "Integrated combination
matrices"). Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it. The GPU library shares no code with it and never
calls it.

Reductions (sum, mean, std, max, min of PCF collections) and pointwise
combinations of two sets live in ``reduce.py`` (plain Python). The pair
integrals live in ``pcf_oracle.c`` (built with ``gcc -O2 -ffp-contract=off``);
this module only builds that file and marshals NumPy arrays to it through
ctypes. Kinds: ``LP`` (L_p distance), ``LP_POW`` (d_p^p) and ``GRAM`` (L2
inner product); ``entries_ab`` integrates over a range [a, b) (Section 2.2)
and ``entries_w`` with a time weight through the antiderivative H (Section 3);
``single`` gives the single-PCF integrals, L_p norms and sup norms (Section
3.2).

Parity pins: every function here is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against printed values, closed forms, exact rational
arithmetic, an independent brute force and finite differences. The averaging
of one-sided time derivatives at a breakpoint shared by two different PCFs is
pinned by exact one-sided differences of the forward oracle on dyadic data;
the FP32 mode of ``reduce.py`` by float32 NumPy evaluation of the same tree.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

LP, LP_POW, GRAM = 0, 1, 2
S_INTEGRAL, S_NORM, S_NORM_POW, S_NORM_INF = 0, 1, 2, 3
W_EXP, W_POW = 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_F64P = ctypes.POINTER(ctypes.c_double)
_I64P = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (plain C, no GPU)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
             "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_pair.restype = ctypes.c_double
        lib.orc_pair.argtypes = [ctypes.c_int, ctypes.c_double, _F64P, _F64P,
                                 ctypes.c_int64, _F64P, _F64P, ctypes.c_int64,
                                 _F64P]
        lib.orc_entries.restype = ctypes.c_int
        lib.orc_entries.argtypes = [ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int64, _I64P, _F64P, _F64P,
                                    ctypes.c_int64, _I64P, _I64P, _F64P, _F64P]
        lib.orc_matrix.restype = ctypes.c_int
        lib.orc_matrix.argtypes = [ctypes.c_int, ctypes.c_double,
                                   ctypes.c_int64, _I64P, _F64P, _F64P, _F64P]
        lib.orc_backward.restype = ctypes.c_int
        lib.orc_backward.argtypes = [ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int64, _I64P, _F64P, _F64P,
                                     _F64P, _F64P, _F64P]
        lib.orc_entries_ab.restype = ctypes.c_int
        lib.orc_entries_ab.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int64, _I64P, _F64P,
                                       _F64P, ctypes.c_int64, _I64P, _I64P, _F64P,
                                       _F64P]
        lib.orc_entries_w.restype = ctypes.c_int
        lib.orc_entries_w.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int64, _I64P, _F64P, _F64P, ctypes.c_int64,
                                      _I64P, _I64P, _F64P, _F64P]
        lib.orc_single.restype = ctypes.c_int
        lib.orc_single.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int64, _I64P, _F64P,
                                   _F64P, _F64P, _F64P]
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _p(a, typ):
    return a.ctypes.data_as(typ)


def pair(kind, p, tf, vf, tg, vg, with_abs=False):
    """F(f, g) for one pair of PCFs given as time/value arrays."""
    lib = _load()
    tf, vf, tg, vg = _f64(tf), _f64(vf), _f64(tg), _f64(vg)
    ab = ctypes.c_double(0.0)
    r = lib.orc_pair(int(kind), float(p), _p(tf, _F64P), _p(vf, _F64P),
                     len(tf), _p(tg, _F64P), _p(vg, _F64P), len(tg),
                     ctypes.byref(ab))
    return (r, ab.value) if with_abs else r


def entries(kind, p, offsets, t, v, I, J, with_abs=False):
    """F(f_I[k], f_J[k]) for listed ordered pairs of a CSR set.

    ``offsets``/``t``/``v`` are the host CSR arrays (values are promoted to
    float64 exactly, so FP32 data is evaluated on its rounded values).
    """
    lib = _load()
    offsets, t, v = _i64(offsets), _f64(t), _f64(v)
    I, J = _i64(I), _i64(J)
    out = np.empty(len(I), dtype=np.float64)
    ab = np.empty(len(I), dtype=np.float64)
    rc = lib.orc_entries(int(kind), float(p), len(offsets) - 1,
                         _p(offsets, _I64P), _p(t, _F64P), _p(v, _F64P),
                         len(I), _p(I, _I64P), _p(J, _I64P), _p(out, _F64P),
                         _p(ab, _F64P))
    if rc:
        raise ValueError("oracle: bad pair index")
    return (out, ab) if with_abs else out


def entries_ab(kind, p, a, b, offsets, t, v, I, J, with_abs=False):
    """As ``entries`` over the integration range [a, b) (Section 2.2)."""
    lib = _load()
    offsets, t, v = _i64(offsets), _f64(t), _f64(v)
    I, J = _i64(I), _i64(J)
    out = np.empty(len(I), dtype=np.float64)
    ab = np.empty(len(I), dtype=np.float64)
    rc = lib.orc_entries_ab(int(kind), float(p), float(a), float(b), len(offsets) - 1,
                            _p(offsets, _I64P), _p(t, _F64P), _p(v, _F64P), len(I),
                            _p(I, _I64P), _p(J, _I64P), _p(out, _F64P), _p(ab, _F64P))
    if rc:
        raise ValueError("oracle: bad pair index or bounds")
    return (out, ab) if with_abs else out


def entries_w(kind, p, weight, c, offsets, t, v, I, J, a=0.0, b=np.inf, with_abs=False):
    """As ``entries_ab`` with the time weight ``weight`` (``W_EXP``:
    w(t) = exp(-c t); ``W_POW``: w(t) = t^c): the time-dependent h of
    Section 3 summed through its antiderivative H = h0 * W. ``with_abs``
    also returns sum |h0| (|W(r)| + |W(l)|)."""
    lib = _load()
    offsets, t, v = _i64(offsets), _f64(t), _f64(v)
    I, J = _i64(I), _i64(J)
    out = np.empty(len(I), dtype=np.float64)
    ab = np.empty(len(I), dtype=np.float64)
    rc = lib.orc_entries_w(int(kind), float(p), int(weight), float(c), float(a), float(b),
                           len(offsets) - 1, _p(offsets, _I64P), _p(t, _F64P), _p(v, _F64P),
                           len(I), _p(I, _I64P), _p(J, _I64P), _p(out, _F64P), _p(ab, _F64P))
    if rc:
        raise ValueError("oracle: bad pair index, bounds or weight")
    return (out, ab) if with_abs else out


def entries_terms(terms, q, offsets, t, v, I, J):
    """F(f_I[k], f_J[k]) = r(sum_m coef_m I_m) for the time-dependent
    combination h(a, b, t) = sum_m coef_m h0_m(a, b) w_m(t) (Section 3:
    H(a, b, r) - H(a, b, l) per rectangle, H = sum_m coef_m h0_m W_m), by the
    definition: each term's integral (``entries`` / ``entries_w``), the
    coefficients, the sum, then r(x) = x^(1/q) (q = 0: none). ``terms``:
    ``(kind, p, weight, c, coef)`` with kind LP_POW or GRAM, weight 0 (w = 1),
    W_EXP or W_POW."""
    total = np.zeros(len(I), dtype=np.float64)
    for kind, p, weight, c, coef in terms:
        if weight:
            m = entries_w(kind, p, weight, c, offsets, t, v, I, J)
        else:
            m = entries(kind, p, offsets, t, v, I, J)
        total = total + coef * m
    return total ** (1.0 / q) if q else total


def matrix(kind, p, offsets, t, v):
    """The full M x M matrix, every entry computed on its own."""
    lib = _load()
    offsets, t, v = _i64(offsets), _f64(t), _f64(v)
    M = len(offsets) - 1
    out = np.empty((M, M), dtype=np.float64)
    rc = lib.orc_matrix(int(kind), float(p), M, _p(offsets, _I64P),
                        _p(t, _F64P), _p(v, _F64P), _p(out, _F64P))
    if rc:
        raise MemoryError("oracle: allocation failed")
    return out


def backward(kind, p, offsets, t, v, G):
    """dL/dt, dL/dv for L = sum_ij G_ij F(f_i, f_j) (CSR layout)."""
    lib = _load()
    offsets, t, v = _i64(offsets), _f64(t), _f64(v)
    M = len(offsets) - 1
    G = _f64(G).reshape(M, M)
    gt = np.zeros(len(t), dtype=np.float64)
    gv = np.zeros(len(v), dtype=np.float64)
    rc = lib.orc_backward(int(kind), float(p), M, _p(offsets, _I64P),
                          _p(t, _F64P), _p(v, _F64P), _p(G, _F64P),
                          _p(gt, _F64P), _p(gv, _F64P))
    if rc:
        raise MemoryError("oracle: allocation failed")
    return gt, gv


def single(kind, p, a, b, offsets, t, v, with_abs=False):
    """F(f_i) = r(int_a^b h(f_i)) for every PCF of a CSR set (Section 3.2,
    segment iteration); ``b`` may be ``inf``."""
    lib = _load()
    offsets, t, v = _i64(offsets), _f64(t), _f64(v)
    n = len(offsets) - 1
    out = np.empty(n, dtype=np.float64)
    ab = np.empty(n, dtype=np.float64)
    rc = lib.orc_single(int(kind), float(p), float(a), float(b), n, _p(offsets, _I64P),
                        _p(t, _F64P), _p(v, _F64P), _p(out, _F64P), _p(ab, _F64P))
    if rc:
        raise ValueError("oracle: need 0 <= a < b")
    return (out, ab) if with_abs else out

