"""Pins of the oracle's time-weighted pair integrals (Section 2.2, weighted
L_p and inner product; Section 3, a time-dependent h summed through its
antiderivative H): closed forms worked by hand, the constant weight against
the unweighted oracle, adaptive quadrature of the weighted integrand
(SciPy, breakpoints given), additivity over the range and the change of
variables tau = W(t)."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_2404_07183_amd import workloads

INF = math.inf
E = math.exp


def _set(*pcfs):
    o = np.concatenate([[0], np.cumsum([len(t) for t, _ in pcfs])])
    return (o, np.concatenate([np.asarray(t, float) for t, _ in pcfs]),
            np.concatenate([np.asarray(v, float) for _, v in pcfs]))


def _w(kind, p, wk, c, o, t, v, a=0.0, b=INF, i=0, j=1):
    return oracle.entries_w(kind, p, wk, c, o, t, v, [i], [j], a=a, b=b)[0]


def test_closed_forms():
    # f = 2 on [0,1), -3 on [1,4); g = 1 on [0,2); both 0 afterwards
    o, t, v = _set(([0.0, 1.0, 4.0], [2.0, -3.0, 0.0]), ([0.0, 2.0], [1.0, 0.0]))
    # w(t) = e^{-t}: int_l^r w = e^{-l} - e^{-r}
    seg = lambda l, r: E(-l) - E(-r)
    l1 = 1 * seg(0, 1) + 4 * seg(1, 2) + 3 * seg(2, 4)
    assert _w(oracle.LP, 1.0, oracle.W_EXP, 1.0, o, t, v) == pytest.approx(l1, rel=1e-15)
    d2 = 1 * seg(0, 1) + 16 * seg(1, 2) + 9 * seg(2, 4)
    assert _w(oracle.LP_POW, 2.0, oracle.W_EXP, 1.0, o, t, v) == pytest.approx(d2, rel=1e-15)
    assert _w(oracle.LP, 2.0, oracle.W_EXP, 1.0, o, t, v) == pytest.approx(math.sqrt(d2), rel=1e-15)
    gr = 2 * seg(0, 1) - 3 * seg(1, 2)
    assert _w(oracle.GRAM, 0.0, oracle.W_EXP, 1.0, o, t, v) == pytest.approx(gr, rel=1e-14)
    # w(t) = t: int_l^r w = (r^2 - l^2) / 2, over [0.5, 3)
    q = lambda l, r: (r * r - l * l) / 2
    l1p = 1 * q(0.5, 1) + 4 * q(1, 2) + 3 * q(2, 3)
    assert _w(oracle.LP, 1.0, oracle.W_POW, 1.0, o, t, v, a=0.5, b=3.0) == pytest.approx(l1p, rel=1e-15)
    # w(t) = t^{-1/2} (integrable at 0): int_l^r w = 2 (sqrt r - sqrt l)
    s = lambda l, r: 2 * (math.sqrt(r) - math.sqrt(l))
    gr2 = 2 * s(0, 1) - 3 * s(1, 2)
    assert _w(oracle.GRAM, 0.0, oracle.W_POW, -0.5, o, t, v) == pytest.approx(gr2, rel=1e-14)
    # a PCF against itself: zero distance for any weight
    assert _w(oracle.LP, 1.0, oracle.W_EXP, 3.0, o, t, v, i=0, j=0) == 0.0
    with pytest.raises(ValueError):
        _w(oracle.LP, 1.0, oracle.W_EXP, 0.0, o, t, v)  # c must be > 0
    with pytest.raises(ValueError):
        _w(oracle.LP, 1.0, oracle.W_POW, -1.0, o, t, v)  # c must be > -1


@pytest.mark.parametrize("kind,p", [(oracle.LP, 1.0), (oracle.LP, 2.5), (oracle.GRAM, 0.0)])
def test_constant_weight_is_unweighted(kind, p):
    o, t, v = workloads.uniform_counts(25, 1, 30, seed=71)
    I, J = np.meshgrid(np.arange(25), np.arange(25), indexing="ij")
    I, J = I.ravel(), J.ravel()
    for a, b in ((0.0, INF), (1.5, 9.0)):
        wv, ab = oracle.entries_w(kind, p, oracle.W_POW, 0.0, o, t, v, I, J, a=a, b=b,
                                  with_abs=True)
        uv = oracle.entries_ab(kind, p, a, b, o, t, v, I, J)
        sc = ab if (kind != oracle.LP or p == 1.0) else ab ** (1.0 / p)
        assert np.all(np.abs(wv - uv) <= 1e-13 * np.maximum(sc, 1e-300))


def _pcf_at(ts, vs, x):
    return vs[np.searchsorted(ts, x, side="right") - 1]


@pytest.mark.parametrize("wk,c,a", [(oracle.W_EXP, 0.7, 0.0), (oracle.W_EXP, 3.0, 0.4),
                                    (oracle.W_POW, 0.5, 0.0), (oracle.W_POW, 2.0, 0.2),
                                    (oracle.W_POW, -0.5, 0.3)])
def test_quadrature(wk, c, a):
    rng = np.random.default_rng(72)
    w = (lambda x: math.exp(-c * x)) if wk == oracle.W_EXP else (lambda x: x ** c)
    for trial in range(6):
        pcfs = []
        for _ in range(2):
            n = int(rng.integers(1, 7))
            ts = np.concatenate([[0.0], np.cumsum(rng.exponential(1.0, n - 1))])
            vs = np.concatenate([rng.standard_normal(n - 1), [0.0]])
            pcfs.append((ts, vs))
        o, t, v = _set(*pcfs)
        (tf, vf), (tg, vg) = pcfs
        end = max(tf[-1], tg[-1], a) + 1.0
        pts = [x for x in np.concatenate([tf, tg]) if a < x < end]
        for kind, p, h in ((oracle.LP_POW, 2.0, lambda x, y: (x - y) ** 2),
                           (oracle.GRAM, 0.0, lambda x, y: x * y)):
            fn = lambda x: h(_pcf_at(tf, vf, x), _pcf_at(tg, vg, x)) * w(x)
            ref, _ = integrate.quad(fn, a, end, points=pts or None, limit=200,
                                    epsabs=1e-13, epsrel=1e-12)
            got = _w(kind, p, wk, c, o, t, v, a=a)
            assert got == pytest.approx(ref, rel=1e-8, abs=1e-10), (trial, kind)


def test_additivity_and_change_of_variables():
    o, t, v = workloads.uniform_counts(12, 1, 25, seed=73)
    I, J = np.meshgrid(np.arange(12), np.arange(12), indexing="ij")
    I, J = I.ravel(), J.ravel()
    for wk, c in ((oracle.W_EXP, 0.3), (oracle.W_POW, 1.5)):
        for kind in (oracle.LP_POW, oracle.GRAM):
            whole, ab = oracle.entries_w(kind, 2.0, wk, c, o, t, v, I, J, a=0.5, b=12.0,
                                         with_abs=True)
            left = oracle.entries_w(kind, 2.0, wk, c, o, t, v, I, J, a=0.5, b=4.0)
            right = oracle.entries_w(kind, 2.0, wk, c, o, t, v, I, J, a=4.0, b=12.0)
            assert np.all(np.abs(whole - (left + right)) <= 1e-13 * np.maximum(ab, 1e-300))
        # tau = W(t): the weighted integral over [0, inf) is the plain integral
        # of the PCFs carried to the tau axis (W strictly increasing)
        W = (lambda x: -np.expm1(-c * x) / c) if wk == oracle.W_EXP else \
            (lambda x: x ** (c + 1) / (c + 1))
        for kind, p in ((oracle.LP, 1.0), (oracle.GRAM, 0.0)):
            wv, ab = oracle.entries_w(kind, p, wk, c, o, t, v, I, J, with_abs=True)
            uv = oracle.entries(kind, p, o, W(t), v, I, J)
            assert np.all(np.abs(wv - uv) <= 1e-13 * np.maximum(ab, 1e-300))
