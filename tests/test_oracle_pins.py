"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the pin it provides. None of them re-types the oracle's own
formula: they use printed values (the user guide's matrices, Figure 1's
rectangles), closed forms for step functions, exact dense resampling on a
dyadic grid (the integrand is constant on every grid cell, so a midpoint sum is
exact), invariants (metric axioms, polarisation, refinement and scaling
invariance) and an independent NumPy union-grid evaluation.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _csr(pcfs):
    offsets = [0]
    t, v = [], []
    for rows in pcfs:
        for tt, vv in rows:
            t.append(float(tt))
            v.append(float(vv))
        offsets.append(len(t))
    return (np.array(offsets, dtype=np.int64), np.array(t), np.array(v))


def _rand_pcf(rng, n, dyadic=False, grid=4, tmax=40):
    """Random PCF with n rows, last value 0. Dyadic: times on a 1/grid grid
    and values small multiples of 1/4 (every product and sum exact)."""
    if dyadic:
        ticks = np.sort(rng.choice(np.arange(1, tmax), size=n - 1, replace=False))
        t = np.concatenate([[0.0], ticks / grid])
        v = rng.integers(-8, 9, size=n) / 4.0
    else:
        t = np.concatenate([[0.0], np.cumsum(rng.exponential(1.0, size=n - 1))])
        v = rng.standard_normal(size=n)
    v[-1] = 0.0
    return t, v


# --------------------------------------------------------------------- P1
def test_userguide_printed_matrices():
    """P1: Section 5.2 prints the L1, L3.5 and Gram matrices of four PCFs."""
    g = json.load(open(os.path.join(GOLD, "userguide_4pcf.json")))
    o, t, v = _csr(g["pcfs"])
    assert np.array_equal(oracle.matrix(oracle.LP, 1.0, o, t, v),
                          np.array(g["l1"], dtype=float))
    assert np.array_equal(oracle.matrix(oracle.GRAM, 0.0, o, t, v),
                          np.array(g["gram"], dtype=float))
    m35 = oracle.matrix(oracle.LP, 3.5, o, t, v)
    half_ulp_print = 0.5 * 10.0 ** (-g["l3_5_decimals"])
    assert np.max(np.abs(m35 - np.array(g["l3_5"]))) <= half_ulp_print + 1e-15


# --------------------------------------------------------------------- P2
def test_figure1_rectangles():
    """P2: the rectangles drawn in Figure 1 give d_1, d_2^2 and <f,g>."""
    g = json.load(open(os.path.join(GOLD, "figure1_rectangles.json")))
    f = np.array(g["f"], dtype=float)
    h = np.array(g["g"], dtype=float)
    rects = g["rectangles"]
    l1 = sum(abs(a - b) * (r - l) for l, r, a, b in rects)
    l2 = sum((a - b) ** 2 * (r - l) for l, r, a, b in rects)
    ip = sum(a * b * (r - l) for l, r, a, b in rects)
    assert (l1, l2, ip) == (7, 11, 24)
    assert oracle.pair(oracle.LP, 1.0, f[:, 0], f[:, 1], h[:, 0], h[:, 1]) == l1
    assert oracle.pair(oracle.LP_POW, 2.0, f[:, 0], f[:, 1], h[:, 0], h[:, 1]) == l2
    assert oracle.pair(oracle.LP, 2.0, f[:, 0], f[:, 1], h[:, 0], h[:, 1]) == math.sqrt(l2)
    assert oracle.pair(oracle.GRAM, 0.0, f[:, 0], f[:, 1], h[:, 0], h[:, 1]) == ip
    # the rectangles tile [0, 5) without gaps, in time order
    assert [r[0] for r in rects[1:]] == [r[1] for r in rects[:-1]]


# --------------------------------------------------------------------- P3
@pytest.mark.parametrize("seed", range(20))
def test_step_function_closed_forms(seed):
    """P3: f = c on [0,a), g = d on [0,b), a <= b (both then 0):
    d_1 = |c-d| a + |d| (b-a); d_2^2 = (c-d)^2 a + d^2 (b-a); <f,g> = c d a."""
    rng = np.random.default_rng(seed)
    a, b = np.sort(rng.integers(1, 64, size=2) / 8.0)
    if a == b:
        b = a + 0.5
    c, d = rng.integers(-20, 21, size=2) / 4.0
    tf, vf = np.array([0.0, a]), np.array([c, 0.0])
    tg, vg = np.array([0.0, b]), np.array([d, 0.0])
    for (F, G) in [((tf, vf), (tg, vg)), ((tg, vg), (tf, vf))]:
        args = (*F, *G)
        assert oracle.pair(oracle.LP, 1.0, *args) == abs(c - d) * a + abs(d) * (b - a)
        assert oracle.pair(oracle.LP_POW, 2.0, *args) == (c - d) ** 2 * a + d * d * (b - a)
        assert oracle.pair(oracle.GRAM, 0.0, *args) == c * d * a
        p = 3.0
        exp = abs(c - d) ** p * a + abs(d) ** p * (b - a)
        assert oracle.pair(oracle.LP_POW, p, *args) == pytest.approx(exp, rel=1e-14, abs=1e-300)


# ----------------------------------------------------------------- P4 / P9
def _dense_resample(kind, p, tf, vf, tg, vg, grid):
    """Exact integral by dense resampling: all breakpoints are multiples of
    1/grid, so f and g are constant on each cell [k/grid, (k+1)/grid); sample
    at cell midpoints (np.searchsorted evaluates the PCFs) and add in exact
    rational arithmetic. Beyond the last breakpoint both are constant."""
    T = max(tf[-1], tg[-1])
    ncell = int(round(T * grid))
    mids = (np.arange(ncell) + 0.5) / grid
    fv = vf[np.searchsorted(tf, mids, side="right") - 1]
    gv = vg[np.searchsorted(tg, mids, side="right") - 1]
    total = Fraction(0)
    w = Fraction(1, grid)
    for a, b in zip(fv, gv):
        a, b = Fraction(a), Fraction(b)
        if kind == oracle.GRAM:
            hv = a * b
        else:
            hv = abs(a - b) ** int(p)
        total += hv * w
    return total


@pytest.mark.parametrize("seed", range(12))
def test_dense_resampling_exact_dyadic(seed):
    """P4/P9: on dyadic data every width, product and partial sum is exact in
    FP64, so the oracle must equal the exact rational integral bit for bit."""
    rng = np.random.default_rng(100 + seed)
    nf, ng = rng.integers(1, 12, size=2)
    tf, vf = _rand_pcf(rng, nf, dyadic=True)
    tg, vg = _rand_pcf(rng, ng, dyadic=True)
    for kind, p in [(oracle.LP, 1.0), (oracle.LP_POW, 2.0), (oracle.GRAM, 0.0),
                    (oracle.LP_POW, 3.0)]:
        exact = _dense_resample(kind, p, tf, vf, tg, vg, grid=4)
        assert oracle.pair(kind, p, tf, vf, tg, vg) == float(exact)


@pytest.mark.parametrize("seed", range(8))
def test_oracle_error_within_rounding_bound(seed):
    """P9: on non-dyadic data the FP64 result is within the textbook bound of
    left-to-right summation, 2 q u sum|terms| (q cells, u = 2^-53), of the
    exact rational value of the same (rounded) inputs."""
    rng = np.random.default_rng(200 + seed)
    tf, vf = _rand_pcf(rng, int(rng.integers(2, 30)))
    tg, vg = _rand_pcf(rng, int(rng.integers(2, 30)))
    # exact value: union grid in rationals
    grid = sorted(set(Fraction(x) for x in tf) | set(Fraction(x) for x in tg))
    tfF = [Fraction(x) for x in tf]
    tgF = [Fraction(x) for x in tg]

    def val(ts, vs, x):
        k = max(i for i in range(len(ts)) if ts[i] <= x)
        return Fraction(vs[k])

    for kind, p in [(oracle.LP, 1.0), (oracle.LP_POW, 2.0), (oracle.GRAM, 0.0)]:
        tot = Fraction(0)
        tot_abs = Fraction(0)
        for l, r in zip(grid[:-1], grid[1:]):
            a, b = val(tfF, vf, l), val(tgF, vg, l)
            hv = a * b if kind == oracle.GRAM else abs(a - b) ** int(p)
            tot += hv * (r - l)
            tot_abs += abs(hv * (r - l))
        got = oracle.pair(kind, p, tf, vf, tg, vg)
        q = len(grid)
        assert abs(Fraction(got) - tot) <= 3 * q * Fraction(2) ** -53 * tot_abs


# --------------------------------------------------------------------- P7
def _numpy_union_grid(kind, p, tf, vf, tg, vg):
    """Independent evaluation: np.union1d builds the common discretization,
    np.searchsorted evaluates both PCFs on it, np.sum adds the cells."""
    s = np.union1d(tf, tg)
    fv = vf[np.searchsorted(tf, s, side="right") - 1]
    gv = vg[np.searchsorted(tg, s, side="right") - 1]
    hv = fv * gv if kind == oracle.GRAM else np.abs(fv - gv) ** p
    return float(np.sum(hv[:-1] * np.diff(s)))


@pytest.mark.parametrize("seed", range(10))
def test_numpy_union_grid(seed):
    """P7: random continuous data vs the independent NumPy evaluation."""
    rng = np.random.default_rng(300 + seed)
    tf, vf = _rand_pcf(rng, int(rng.integers(1, 200)))
    tg, vg = _rand_pcf(rng, int(rng.integers(1, 200)))
    for kind, p in [(oracle.LP_POW, 1.0), (oracle.LP_POW, 2.0), (oracle.GRAM, 0.0),
                    (oracle.LP_POW, 3.5)]:
        got, ab = oracle.pair(kind, p, tf, vf, tg, vg, with_abs=True)
        ref = _numpy_union_grid(kind, p, tf, vf, tg, vg)
        assert abs(got - ref) <= 1e-13 * max(ab, 1e-300)


@pytest.mark.parametrize("seed", range(10))
def test_refinement_invariance(seed):
    """P7 (Section 2, refinement): inserting extra breakpoints that repeat
    the current value leaves every integral unchanged (exact, dyadic data)."""
    rng = np.random.default_rng(400 + seed)
    tf, vf = _rand_pcf(rng, int(rng.integers(1, 10)), dyadic=True, grid=8, tmax=60)
    tg, vg = _rand_pcf(rng, int(rng.integers(1, 10)), dyadic=True, grid=8, tmax=60)
    extra = np.setdiff1d(np.arange(1, 80) / 8.0, tf)
    extra = rng.choice(extra, size=min(5, len(extra)), replace=False)
    tr = np.sort(np.concatenate([tf, extra]))
    vr = vf[np.searchsorted(tf, tr, side="right") - 1]
    for kind, p in [(oracle.LP, 1.0), (oracle.LP_POW, 2.0), (oracle.GRAM, 0.0)]:
        assert oracle.pair(kind, p, tf, vf, tg, vg) == oracle.pair(kind, p, tr, vr, tg, vg)


# --------------------------------------------------------------- P5 / P6
def test_metric_axioms_and_polarisation():
    """P5: d(f,f) = 0, symmetry, d >= 0, triangle inequality.
    P6: d_2^2 = <f,f> + <g,g> - 2<f,g> within rounding."""
    rng = np.random.default_rng(7)
    pcfs = []
    for _ in range(12):
        t, v = _rand_pcf(rng, int(rng.integers(1, 40)))
        pcfs.append(list(zip(t, v)))
    o, t, v = _csr(pcfs)
    for p in (1.0, 2.0, 3.5):
        D = oracle.matrix(oracle.LP, p, o, t, v)
        assert np.all(np.diag(D) == 0.0)
        assert np.array_equal(D, D.T)
        assert np.all(D >= 0)
        M = len(D)
        for i in range(M):
            for j in range(M):
                assert np.all(D[i, j] <= D[i, :] + D[:, j] + 1e-12 * (1 + D[i, j]))
    G = oracle.matrix(oracle.GRAM, 0.0, o, t, v)
    D2 = oracle.matrix(oracle.LP_POW, 2.0, o, t, v)
    dg = np.diag(G)
    pol = dg[:, None] + dg[None, :] - 2 * G
    scale = dg[:, None] + dg[None, :]
    assert np.all(np.abs(D2 - pol) <= 1e-12 * scale + 1e-300)


# --------------------------------------------------------------------- P8
@pytest.mark.parametrize("seed", range(6))
def test_scaling(seed):
    """P8: values x 2^a scale d_p by 2^a and <,> by 2^(2a); times x 2^b scale
    d_p^p and <,> by 2^b. Powers of two make both exact."""
    rng = np.random.default_rng(500 + seed)
    tf, vf = _rand_pcf(rng, int(rng.integers(2, 50)))
    tg, vg = _rand_pcf(rng, int(rng.integers(2, 50)))
    a, b = 3, -2
    sa, sb = 2.0 ** a, 2.0 ** b
    for kind, p in [(oracle.LP, 1.0), (oracle.LP_POW, 2.0), (oracle.GRAM, 0.0)]:
        base = oracle.pair(kind, p, tf, vf, tg, vg)
        vs = oracle.pair(kind, p, tf, vf * sa, tg, vg * sa)
        ts = oracle.pair(kind, p, tf * sb, vf, tg * sb, vg)
        vpow = 2 if kind == oracle.GRAM else p
        assert vs == base * sa ** vpow
        assert ts == base * sb


# ------------------------------------------------------ contract handling
def test_tail_rule_and_contract():
    """Reading of the unbounded last cell: 0 when h of the last values is 0,
    an infinity otherwise; contract violations give NaN."""
    t = np.array([0.0, 1.0])
    assert oracle.pair(oracle.LP, 1.0, t, np.array([1.0, 0.0]), t, np.array([2.0, 0.0])) == 1.0
    assert oracle.pair(oracle.LP, 1.0, t, np.array([1.0, 1.0]), t, np.array([2.0, 0.0])) == math.inf
    assert oracle.pair(oracle.LP, 1.0, t, np.array([1.0, 3.0]), t, np.array([2.0, 3.0])) == 1.0
    assert oracle.pair(oracle.GRAM, 0.0, t, np.array([1.0, -1.0]), t, np.array([2.0, 1.0])) == -math.inf
    assert math.isnan(oracle.pair(oracle.LP, 1.0, np.array([0.5, 1.0]), np.array([1.0, 0.0]),
                                  t, np.array([1.0, 0.0])))
    assert math.isnan(oracle.pair(oracle.LP, 1.0, np.array([0.0, 1.0, 1.0]), np.array([1.0, 2.0, 0.0]),
                                  t, np.array([1.0, 0.0])))
    # one-row PCFs: the constant (zero) function
    z = np.array([0.0])
    assert oracle.pair(oracle.LP, 1.0, z, np.array([0.0]), t, np.array([2.0, 0.0])) == 2.0
    assert oracle.pair(oracle.GRAM, 0.0, z, np.array([0.0]), z, np.array([0.0])) == 0.0
