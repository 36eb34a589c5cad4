"""Pins of the reductions oracle (Section 2.1 reductions, Section 4
Algorithm ReducePair and reduction trees): pointwise NumPy evaluation of the
mean, extremes and sample standard deviation at every breakpoint and between
them, exactness on dyadic data, the minimal-representation invariants, a
worked two-PCF example and the single-PCF group."""
import math

import numpy as np
import pytest

from oracle import reduce as red
from paper_2404_07183_amd import workloads


def _probe_points(offsets, t):
    b = np.unique(t)
    mids = (b[:-1] + b[1:]) / 2 if len(b) > 1 else b
    return np.concatenate([b, mids, [b[-1] + 1.0]])


def _values(offsets, t, v, lo, hi, x):
    return np.stack([red.evaluate((t[offsets[i]:offsets[i + 1]], v[offsets[i]:offsets[i + 1]]), x)
                     for i in range(lo, hi)])


def _check_minimal(pcf):
    t, v = pcf
    assert t[0] == 0.0 and np.all(np.diff(t) > 0)
    assert np.all(v[1:] != v[:-1])


def test_worked_example():
    # f = 2 on [0,1), -3 on [1,4); g = 1 on [0,2), 2 on [2,3); zero afterwards
    f = (np.array([0.0, 1.0, 4.0]), np.array([2.0, -3.0, 0.0]))
    g = (np.array([0.0, 2.0, 3.0]), np.array([1.0, 2.0, 0.0]))
    s = red.reduce_pair(f, g, red.OPS["sum"])
    assert s[0].tolist() == [0.0, 1.0, 2.0, 3.0, 4.0]
    assert s[1].tolist() == [3.0, -2.0, -1.0, -3.0, 0.0]
    m = red.reduce_pair(f, g, red.OPS["max"])  # the run of 0 from t = 3 is one row
    assert m[0].tolist() == [0.0, 1.0, 2.0, 3.0] and m[1].tolist() == [2.0, 1.0, 2.0, 0.0]
    n = red.reduce_pair(f, g, red.OPS["min"])
    assert n[0].tolist() == [0.0, 1.0, 4.0] and n[1].tolist() == [1.0, -3.0, 0.0]
    # std of {f, g}: |f - g| / sqrt(2) pointwise
    o = np.array([0, 3, 6])
    t = np.concatenate([f[0], g[0]])
    v = np.concatenate([f[1], g[1]])
    (st, sv), = red.reduce_groups("std", [0, 2], o, t, v)
    x = _probe_points(o, t)
    want = np.abs(red.evaluate(f, x) - red.evaluate(g, x)) / math.sqrt(2)
    assert np.allclose(red.evaluate((st, sv), x), want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("op", ["sum", "mean", "max", "min", "std"])
def test_pointwise(op):
    o, t, v = workloads.uniform_counts(37, 1, 40, seed=91)
    groups = [0, 1, 2, 9, 20, 37]
    if op == "std":
        groups = [0, 2, 9, 20, 37]
    res = red.reduce_groups(op, groups, o, t, v)
    x = _probe_points(o, t)
    for b, pcf in enumerate(res):
        vals = _values(o, t, v, groups[b], groups[b + 1], x)
        want = {"sum": lambda a: a.sum(0), "mean": lambda a: a.mean(0),
                "max": lambda a: a.max(0), "min": lambda a: a.min(0),
                "std": lambda a: a.std(0, ddof=1)}[op](vals)
        got = red.evaluate(pcf, x)
        scale = np.abs(vals).sum(0) + 1e-300
        if op in ("max", "min"):
            assert np.array_equal(got, want)
        elif op == "std":
            # the square root halves relative error; compare the variances
            assert np.all(np.abs(got ** 2 - want ** 2) <= 1e-13 * (scale ** 2 + want ** 2))
        else:
            assert np.all(np.abs(got - want) <= 1e-14 * scale)
        if groups[b + 1] - groups[b] > 1:
            _check_minimal(pcf)
        assert pcf[1][-1] == 0.0  # every f_i ends at 0


def test_dyadic_sums_are_exact():
    rng = np.random.default_rng(92)
    pcfs = []
    for _ in range(23):
        n = int(rng.integers(1, 12))
        ts = np.concatenate([[0.0], np.sort(rng.choice(np.arange(1, 200), n - 1, replace=False))]) / 8
        vs = np.concatenate([rng.integers(-64, 64, n - 1) / 16.0, [0.0]])
        pcfs.append((ts, vs))
    o = np.concatenate([[0], np.cumsum([len(p[0]) for p in pcfs])])
    t = np.concatenate([p[0] for p in pcfs])
    v = np.concatenate([p[1] for p in pcfs])
    (st, sv), = red.reduce_groups("sum", [0, 23], o, t, v)
    x = _probe_points(o, t)
    assert np.array_equal(red.evaluate((st, sv), x), _values(o, t, v, 0, 23, x).sum(0))
    _check_minimal((st, sv))


def test_single_pcf_group_and_pairs():
    # a one-PCF reduction is the PCF itself, rows included; a pair goes
    # through ReducePair, which merges equal neighbours
    f = (np.array([0.0, 1.0, 2.0, 3.0]), np.array([5.0, 5.0, -1.0, 0.0]))
    o = np.array([0, 4, 8])
    t, v = np.concatenate([f[0], f[0]]), np.concatenate([f[1], f[1]])
    (t1, v1), = red.reduce_groups("mean", [0, 1], o, t, v)
    assert t1.tolist() == f[0].tolist() and v1.tolist() == f[1].tolist()
    (t2, v2), = red.reduce_groups("mean", [0, 2], o, t, v)
    assert t2.tolist() == [0.0, 2.0, 3.0] and v2.tolist() == [5.0, -1.0, 0.0]
    with pytest.raises(ValueError):
        red.reduce_groups("std", [0, 1], o, t, v)


@pytest.mark.parametrize("op", ["sum", "sub", "mul", "max", "min", "sqdiff"])
def test_combinations_pointwise(op):
    xs = workloads.uniform_counts(30, 1, 40, seed=93)
    ys = workloads.uniform_counts(30, 1, 40, seed=94)
    res = red.combine_sets(op, xs, ys)
    f = {"sum": np.add, "sub": np.subtract, "mul": np.multiply, "max": np.maximum,
         "min": np.minimum, "sqdiff": lambda a, b: (a - b) ** 2}[op]
    for i, pcf in enumerate(res):
        fi = (xs[1][xs[0][i]:xs[0][i + 1]], xs[2][xs[0][i]:xs[0][i + 1]])
        gi = (ys[1][ys[0][i]:ys[0][i + 1]], ys[2][ys[0][i]:ys[0][i + 1]])
        x = np.unique(np.concatenate([fi[0], gi[0]]))
        x = np.concatenate([x, (x[:-1] + x[1:]) / 2, [x[-1] + 1]])
        assert np.array_equal(red.evaluate(pcf, x), f(red.evaluate(fi, x), red.evaluate(gi, x)))
        _check_minimal(pcf)


def _tree32(vals, op):
    """Level-by-level binary tree over float32 arrays (neighbours (2j, 2j+1),
    an unpaired last item moves up), one NumPy float32 operation per node."""
    level = list(vals)
    while len(level) > 1:
        nxt = [op(level[k], level[k + 1]) for k in range(0, len(level) - 1, 2)]
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    return level[0]


@pytest.mark.parametrize("op", ["sum", "mean", "max", "min", "std"])
def test_pointwise_float32(op):
    """The FP32 mode: every row of the reduced PCF equals, bit for bit, a
    float32 NumPy evaluation of the same tree at every breakpoint and between
    them (each node one float32 add, max or min; mean one float32 division;
    std the float32 squared differences from that mean, tree-summed, divided
    by n - 1 and square-rooted in float32)."""
    f32 = np.float32
    o, t, v = workloads.uniform_counts(41, 1, 40, seed=95, dtype=np.float32)
    assert t.dtype == np.float32 and v.dtype == np.float32
    groups = [0, 2, 4, 10, 25, 41] if op == "std" else [0, 2, 3, 10, 25, 41]
    res = red.reduce_groups(op, groups, o, t, v, dtype=np.float32)
    x = _probe_points(o, t)
    for b, pcf in enumerate(res):
        assert pcf[0].dtype == np.float32 and pcf[1].dtype == np.float32
        vals = [red.evaluate((t[o[i]:o[i + 1]], v[o[i]:o[i + 1]]), x).astype(f32)
                for i in range(groups[b], groups[b + 1])]
        n = len(vals)
        if op in ("max", "min"):
            want = _tree32(vals, np.maximum if op == "max" else np.minimum)
        else:
            s = _tree32(vals, np.add)
            want = s
            if op in ("mean", "std"):
                want = (s / f32(n)).astype(f32)
            if op == "std":
                m = want
                sq = [((a - m) * (a - m)).astype(f32) for a in vals]
                want = np.sqrt((_tree32(sq, np.add) / f32(n - 1)).astype(f32))
        assert want.dtype == np.float32
        got = red.evaluate(pcf, x)
        assert np.array_equal(got, want), (op, b)
        if n > 1:
            _check_minimal(pcf)


@pytest.mark.parametrize("op", ["sum", "sub", "mul", "max", "min", "sqdiff"])
def test_combinations_float32(op):
    """FP32 combinations equal a float32 NumPy evaluation of h(f_i(x), g_i(x))
    at every breakpoint and between them, bit for bit."""
    f32 = np.float32
    xs = workloads.uniform_counts(25, 1, 40, seed=96, dtype=np.float32)
    ys = workloads.uniform_counts(25, 1, 40, seed=97, dtype=np.float32)
    res = red.combine_sets(op, xs, ys, dtype=np.float32)
    f = {"sum": np.add, "sub": np.subtract, "mul": np.multiply, "max": np.maximum,
         "min": np.minimum, "sqdiff": lambda a, b: (a - b) * (a - b)}[op]
    for i, pcf in enumerate(res):
        fi = (xs[1][xs[0][i]:xs[0][i + 1]], xs[2][xs[0][i]:xs[0][i + 1]])
        gi = (ys[1][ys[0][i]:ys[0][i + 1]], ys[2][ys[0][i]:ys[0][i + 1]])
        x = np.unique(np.concatenate([fi[0], gi[0]])).astype(np.float64)
        x = np.concatenate([x, (x[:-1] + x[1:]) / 2, [x[-1] + 1]])
        want = f(red.evaluate(fi, x).astype(f32), red.evaluate(gi, x).astype(f32))
        assert want.dtype == np.float32
        assert np.array_equal(red.evaluate(pcf, x), want)
        _check_minimal(pcf)


def test_dyadic_float32_sums_are_exact():
    """On dyadic FP32 data every float32 partial sum is exact: the FP32
    reduction equals the exact (FP64) pointwise sum."""
    rng = np.random.default_rng(98)
    pcfs = []
    for _ in range(19):
        n = int(rng.integers(1, 12))
        ts = np.concatenate([[0.0], np.sort(rng.choice(np.arange(1, 200), n - 1, replace=False))]) / 8
        vs = np.concatenate([rng.integers(-64, 64, n - 1) / 16.0, [0.0]])
        pcfs.append((ts.astype(np.float32), vs.astype(np.float32)))
    o = np.concatenate([[0], np.cumsum([len(p[0]) for p in pcfs])])
    t = np.concatenate([p[0] for p in pcfs])
    v = np.concatenate([p[1] for p in pcfs])
    (st, sv), = red.reduce_groups("sum", [0, 19], o, t, v, dtype=np.float32)
    x = _probe_points(o, t.astype(np.float64))
    exact = _values(o, t.astype(np.float64), v.astype(np.float64), 0, 19, x).sum(0)
    assert np.array_equal(red.evaluate((st, sv), x).astype(np.float64), exact)
