"""Pins of the oracle's time-dependent combinations given as sums of
separable terms (Section 3: a time-dependent h with a known antiderivative H
in t adds H(a, b, r) - H(a, b, l) per rectangle): adaptive quadrature (SciPy,
breakpoints given) of the integrand h(f(t), g(t), t) for h that are not
separable, a single term against the one-weight oracle, and linearity in the
coefficients."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_2404_07183_amd import workloads


def _pcf_at(ts, vs, x):
    k = int(np.searchsorted(ts, x, side="right")) - 1
    return vs[k]


def _h(terms, a, b, x):
    s = 0.0
    for kind, p, wk, c, coef in terms:
        h0 = abs(a - b) ** p if kind == oracle.LP_POW else a * b
        w = 1.0 if not wk else (math.exp(-c * x) if wk == oracle.W_EXP else x ** c)
        s += coef * h0 * w
    return s


CASES = [
    # |a - b|^2 e^{-0.5 t} + 0.3 a b t^{1/2}: not a product h0(a, b) w(t)
    ([(oracle.LP_POW, 2.0, oracle.W_EXP, 0.5, 1.0), (oracle.GRAM, 0.0, oracle.W_POW, 0.5, 0.3)], 0.0),
    # |a - b| + 2 |a - b|^3 e^{-t}, then the square root
    ([(oracle.LP_POW, 1.0, 0, 0.0, 1.0), (oracle.LP_POW, 3.0, oracle.W_EXP, 1.0, 2.0)], 2.0),
    # a b (1 - e^{-2t}) = a b - a b e^{-2t}: a negative coefficient
    ([(oracle.GRAM, 0.0, 0, 0.0, 1.0), (oracle.GRAM, 0.0, oracle.W_EXP, 2.0, -1.0)], 0.0),
]


@pytest.mark.parametrize("terms,q", CASES)
def test_quadrature(terms, q):
    rng = np.random.default_rng(81)
    for trial in range(6):
        pcfs = []
        for _ in range(2):
            n = int(rng.integers(1, 7))
            ts = np.concatenate([[0.0], np.cumsum(rng.exponential(1.0, n - 1))])
            vs = np.concatenate([rng.standard_normal(n - 1), [0.0]])
            pcfs.append((ts, vs))
        o = np.array([0, len(pcfs[0][0]), len(pcfs[0][0]) + len(pcfs[1][0])])
        t = np.concatenate([pcfs[0][0], pcfs[1][0]])
        v = np.concatenate([pcfs[0][1], pcfs[1][1]])
        (tf, vf), (tg, vg) = pcfs
        end = max(tf[-1], tg[-1]) + 1.0  # past both last breakpoints h(0, 0, t) = 0
        pts = [x for x in np.concatenate([tf, tg]) if 0.0 < x < end]
        fn = lambda x: _h(terms, _pcf_at(tf, vf, x), _pcf_at(tg, vg, x), x)
        ref, _ = integrate.quad(fn, 0.0, end, points=pts or None, limit=200, epsabs=1e-13,
                                epsrel=1e-12)
        if q:
            ref = ref ** (1.0 / q)
        got = oracle.entries_terms(terms, q, o, t, v, [0], [1])[0]
        assert got == pytest.approx(ref, rel=1e-8, abs=1e-10), trial


def test_single_term_and_linearity():
    o, t, v = workloads.uniform_counts(9, 1, 20, seed=82)
    I, J = np.meshgrid(np.arange(9), np.arange(9), indexing="ij")
    I, J = I.ravel(), J.ravel()
    one = oracle.entries_terms([(oracle.LP_POW, 2.0, oracle.W_POW, 1.5, 1.0)], 0.0, o, t, v, I, J)
    assert np.array_equal(one, oracle.entries_w(oracle.LP_POW, 2.0, oracle.W_POW, 1.5, o, t, v, I, J))
    plain = oracle.entries_terms([(oracle.LP_POW, 1.0, 0, 0.0, 1.0)], 0.0, o, t, v, I, J)
    assert np.array_equal(plain, oracle.entries(oracle.LP, 1.0, o, t, v, I, J))
    a = [(oracle.GRAM, 0.0, oracle.W_EXP, 0.4, 1.0)]
    b = [(oracle.LP_POW, 2.0, 0, 0.0, 1.0)]
    ga = oracle.entries_terms(a, 0.0, o, t, v, I, J)
    gb = oracle.entries_terms(b, 0.0, o, t, v, I, J)
    both = oracle.entries_terms([(k, p, w, c, 2.5) for k, p, w, c, _ in a] +
                                [(k, p, w, c, -0.5) for k, p, w, c, _ in b], 0.0, o, t, v, I, J)
    assert np.allclose(both, 2.5 * ga - 0.5 * gb, rtol=1e-14, atol=1e-12)
