"""Pins of the oracle's single-PCF functionals (Section 3.2, segment
iteration): closed forms, the pairwise oracle against the zero PCF and
against itself, additivity over the integration bounds, the tail rule."""
import math

import numpy as np
import pytest

import oracle
from paper_2404_07183_amd import workloads

INF = math.inf


def _one(t, v):
    return np.array([0, len(t)]), np.asarray(t, float), np.asarray(v, float)


def test_closed_forms():
    # f = 2 on [0,1), -3 on [1,4), 0 after
    o, t, v = _one([0.0, 1.0, 4.0], [2.0, -3.0, 0.0])
    S = oracle.single
    assert S(oracle.S_INTEGRAL, 1, 0, INF, o, t, v)[0] == -7.0
    assert S(oracle.S_NORM_POW, 1, 0, INF, o, t, v)[0] == 11.0
    assert S(oracle.S_NORM_POW, 2, 0, INF, o, t, v)[0] == 31.0
    assert S(oracle.S_NORM, 2, 0, INF, o, t, v)[0] == math.sqrt(31.0)
    # bounds inside pieces: 2 * 0.5 + (-3) * 1
    assert S(oracle.S_INTEGRAL, 1, 0.5, 2.0, o, t, v)[0] == -2.0
    # a and b in one piece, and past the last breakpoint
    assert S(oracle.S_INTEGRAL, 1, 1.5, 3.5, o, t, v)[0] == -6.0
    assert S(oracle.S_INTEGRAL, 1, 5.0, 9.0, o, t, v)[0] == 0.0
    # b exactly on a breakpoint, a exactly on one
    assert S(oracle.S_INTEGRAL, 1, 1.0, 4.0, o, t, v)[0] == -9.0
    assert S(oracle.S_INTEGRAL, 1, 0.0, 1.0, o, t, v)[0] == 2.0
    # p = 3.5 by hand
    want = 2.0 ** 3.5 * 1 + 3.0 ** 3.5 * 3
    assert abs(S(oracle.S_NORM_POW, 3.5, 0, INF, o, t, v)[0] - want) <= 1e-14 * want


@pytest.mark.parametrize("seed", [1, 2])
def test_norms_are_distances_to_the_zero_pcf(seed):
    # ||f||_p^p = d_p(f, 0)^p and int f^2 = <f, f> by the pairwise oracle
    o, t, v = workloads.uniform_counts(40, 1, 60, seed=seed)
    z_t, z_v = np.array([0.0]), np.array([0.0])
    for p in (1.0, 2.0, 3.5):
        got, ab = oracle.single(oracle.S_NORM_POW, p, 0, INF, o, t, v, with_abs=True)
        for i in range(len(o) - 1):
            a, b = o[i], o[i + 1]
            ref = oracle.pair(oracle.LP_POW, p, t[a:b], v[a:b], z_t, z_v)
            assert abs(got[i] - ref) <= 1e-13 * ab[i]
    got, ab = oracle.single(oracle.S_NORM_POW, 2.0, 0, INF, o, t, v, with_abs=True)
    for i in range(len(o) - 1):
        a, b = o[i], o[i + 1]
        ref = oracle.pair(oracle.GRAM, 0.0, t[a:b], v[a:b], t[a:b], v[a:b])
        assert abs(got[i] - ref) <= 1e-13 * ab[i]


@pytest.mark.parametrize("seed", [3, 4])
def test_additivity_over_bounds(seed):
    o, t, v = workloads.uniform_counts(30, 1, 80, seed=seed)
    rng = np.random.default_rng(seed)
    for _ in range(5):
        a, c, b = np.sort(rng.uniform(0, 60, 3))
        for kind in (oracle.S_INTEGRAL, oracle.S_NORM_POW):
            ac, s1 = oracle.single(kind, 2.0, a, c, o, t, v, with_abs=True)
            cb, s2 = oracle.single(kind, 2.0, c, b, o, t, v, with_abs=True)
            ab_ = oracle.single(kind, 2.0, a, b, o, t, v)
            assert np.all(np.abs(ac + cb - ab_) <= 1e-12 * (s1 + s2) + 1e-300)
        # and the whole line is the sum of [0, b) and [b, inf)
        left = oracle.single(oracle.S_INTEGRAL, 1, 0, b, o, t, v)
        right = oracle.single(oracle.S_INTEGRAL, 1, b, INF, o, t, v)
        whole, sc = oracle.single(oracle.S_INTEGRAL, 1, 0, INF, o, t, v, with_abs=True)
        assert np.all(np.abs(left + right - whole) <= 1e-12 * sc + 1e-300)


def test_tail_rule_and_bad_bounds():
    # a nonzero last value: infinite over [0, inf), finite over a finite range
    o, t, v = _one([0.0, 2.0], [1.0, -0.5])
    assert oracle.single(oracle.S_INTEGRAL, 1, 0, INF, o, t, v)[0] == -INF
    assert oracle.single(oracle.S_NORM_POW, 1, 0, INF, o, t, v)[0] == INF
    assert oracle.single(oracle.S_INTEGRAL, 1, 0, 4.0, o, t, v)[0] == 1.0
    with pytest.raises(ValueError):
        oracle.single(oracle.S_INTEGRAL, 1, 2.0, 2.0, o, t, v)


def test_sup_norm():
    # f = 2 on [0,1), -3 on [1,4), 0 after
    o, t, v = _one([0.0, 1.0, 4.0], [2.0, -3.0, 0.0])
    S = lambda a, b: oracle.single(oracle.S_NORM_INF, 0, a, b, o, t, v)[0]
    assert S(0, INF) == 3.0
    assert S(0, 1.0) == 2.0       # [0, 1) never reaches the -3 piece
    assert S(0.5, 1.0 + 1e-9) == 3.0
    assert S(4.0, 9.0) == 0.0     # past the last breakpoint
    assert S(1.0, 4.0) == 3.0 and S(0.0, 0.5) == 2.0
    # over [0, inf) it is the largest |v| of the rows (NumPy), and over split
    # ranges the larger of the two parts
    o, t, v = workloads.uniform_counts(40, 1, 60, seed=9)
    whole = oracle.single(oracle.S_NORM_INF, 0, 0.0, INF, o, t, v)
    assert np.array_equal(whole, [np.abs(v[o[i]:o[i + 1]]).max() for i in range(40)])
    left = oracle.single(oracle.S_NORM_INF, 0, 0.0, 7.5, o, t, v)
    right = oracle.single(oracle.S_NORM_INF, 0, 7.5, INF, o, t, v)
    assert np.array_equal(np.maximum(left, right), whole)
    # the L_p norm tends to the sup norm on a bounded range
    big = oracle.single(oracle.S_NORM, 64.0, 0.0, 10.0, o, t, v)
    sup = oracle.single(oracle.S_NORM_INF, 0, 0.0, 10.0, o, t, v)
    assert np.all(big <= sup * 10.0 ** (1 / 64) * (1 + 1e-12))
    assert np.all(big >= sup * 0.85)
