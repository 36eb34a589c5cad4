"""GPU parity of the time-weighted pair integrals (Section 3, time-dependent
h with antiderivative H; Section 2.2, weighted L_p and inner product): the
time warp tau = W(t) on the device, then the unchanged pairwise and cross
kernels, against the oracle's per-cell sum of H(r) - H(l).

Bars: FP64 |gpu - oracle| <= 1e-12 * S, S = sum |h0| (|W(r)| + |W(l)|) (the
magnitudes of the terms the oracle adds); for a root r(I) = I^(1/p) the bar
on I is carried through r's derivative. FP32 (inputs rounded to FP32) at
1e-5 * S."""
import math

import numpy as np
import pytest

import oracle
from paper_2404_07183_amd import api, workloads
from paper_2404_07183_amd._lib import PcfError

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
WEIGHTS = [("exp", 0.3, oracle.W_EXP), ("exp", 2.0, oracle.W_EXP),
           ("pow", 0.5, oracle.W_POW), ("pow", -0.5, oracle.W_POW),
           ("pow", 2.0, oracle.W_POW)]
KINDS = {  # name -> (api call, oracle kind, p)
    "l1": (lambda X, w, **k: api.pdist(X, 1.0, weight=w, **k), oracle.LP, 1.0),
    "l2": (lambda X, w, **k: api.pdist(X, 2.0, weight=w, **k), oracle.LP, 2.0),
    "gram": (lambda X, w, **k: api.gram(X, weight=w, **k), oracle.GRAM, 0.0),
    "l3.5pow": (lambda X, w, **k: api.pdist(X, 3.5, power=True, weight=w, **k),
                oracle.LP_POW, 3.5),
}


def _check(got, ref, ab, kind, p, rel):
    """|got - ref| within rel * ab on I, carried through r(I) = I^(1/p)."""
    tol = rel * np.maximum(ab, 1e-300)
    if kind == oracle.LP and p != 1.0:
        # d = I^(1/p): |dd| <= (1/p) I^(1/p - 1) |dI|
        with np.errstate(divide="ignore", over="ignore"):
            tol = tol * (1.0 / p) * np.where(ref > 0, ref, np.inf) ** (1.0 - p)
    err = np.abs(got - ref)
    bad = ~((err <= tol) | (err == 0))
    return bad


def _np_warp_times(t, kind, c):
    return -np.expm1(-c * t) / c if kind == "exp" else t ** (c + 1) / (c + 1)


def test_warp_rows_and_ties():
    o, t, v = workloads.uniform_counts(200, 1, 120, seed=81)
    X = api.PcfSet(o, t, v, device=DEV)
    # weights whose W stays far from saturation on these times: no ties
    for name, c in (("exp", 0.05), ("pow", 0.5), ("pow", -0.5), ("pow", 2.0)):
        Wx = api.warp(X, name, c)
        assert np.array_equal(Wx.offsets_host, o), name
        wt, wv = Wx.t.cpu().numpy(), Wx.v.cpu().numpy()
        assert np.array_equal(wv, v)
        ref = _np_warp_times(t, name, c)
        ref[o[:-1]] = 0.0
        assert np.allclose(wt, ref, rtol=8e-16, atol=0), name
    # rows whose rounded tau ties collapse onto the last row of the run
    o2, t2, v2 = np.array([0, 5]), np.array([0.0, 1.0, 50.0, 60.0, 70.0]), \
        np.array([1.0, 2.0, 3.0, 4.0, 0.0])
    Wx = api.warp(api.PcfSet(o2, t2, v2, device=DEV), "exp", 1.0)
    assert list(Wx.offsets_host) == [0, 3]
    assert np.array_equal(Wx.v.cpu().numpy(), [1.0, 2.0, 0.0])
    wt = Wx.t.cpu().numpy()
    assert wt[0] == 0.0 and wt[2] == 1.0 and wt[1] == pytest.approx(1 - math.exp(-1), rel=1e-15)


@pytest.mark.parametrize("name", sorted(KINDS))
def test_weighted_matrices_fp64(name):
    fn, okind, p = KINDS[name]
    o, t, v = workloads.uniform_counts(100, 1, 150, seed=82)
    X = api.PcfSet(o, t, v, device=DEV)
    I, J = np.meshgrid(np.arange(X.n), np.arange(X.n), indexing="ij")
    for wname, c, wk in WEIGHTS:
        for bounds in (None, (2.5, 40.0)):
            M = fn(X, (wname, c), bounds=bounds).cpu().numpy().ravel()
            a, b = bounds if bounds else (0.0, np.inf)
            ref, ab = oracle.entries_w(okind, p, wk, c, o, t, v, I.ravel(), J.ravel(),
                                       a=a, b=b, with_abs=True)
            bad = _check(M, ref, ab, okind, p, 1e-12)
            assert not bad.any(), (name, wname, c, bounds, np.argwhere(bad)[:5])


def test_weighted_fp32_and_cross():
    o, t, v = workloads.uniform_counts(120, 10, 200, seed=83, dtype=np.float32)
    X = api.PcfSet(o, t, v, device=DEV)
    I, J = np.meshgrid(np.arange(X.n), np.arange(X.n), indexing="ij")
    for wname, c, wk in WEIGHTS[:3]:
        M = api.pdist(X, 1.0, weight=(wname, c)).cpu().numpy().astype(np.float64)
        ref, ab = oracle.entries_w(oracle.LP, 1.0, wk, c, o, t, v, I.ravel(), J.ravel(),
                                   with_abs=True)
        assert not _check(M.ravel(), ref, ab, oracle.LP, 1.0, 1e-5).any(), wname
    # cross-set, range and weight together: the X x Y block of the joint set
    ys = workloads.uniform_counts(30, 10, 200, seed=84)
    Xd = api.PcfSet(*workloads.uniform_counts(50, 10, 200, seed=85), device=DEV)
    xo, xt, xv = Xd.offsets_host, Xd.t.cpu().numpy(), Xd.v.cpu().numpy()
    Y = api.PcfSet(*ys, device=DEV)
    C = api.cross_gram(Xd, Y, bounds=(1.0, 30.0), weight=("exp", 0.1)).cpu().numpy()
    oj = np.concatenate([xo, xo[-1] + ys[0][1:]])
    tj, vj = np.concatenate([xt, ys[1]]), np.concatenate([xv, ys[2]])
    Ic, Jc = np.meshgrid(np.arange(Xd.n), Xd.n + np.arange(Y.n), indexing="ij")
    refc, abc = oracle.entries_w(oracle.GRAM, 0.0, oracle.W_EXP, 0.1, oj, tj, vj,
                                 Ic.ravel(), Jc.ravel(), a=1.0, b=30.0, with_abs=True)
    assert not _check(C.ravel(), refc, abc, oracle.GRAM, 0.0, 1e-12).any()


def test_weight_errors():
    o, t, v = workloads.uniform_counts(10, 1, 20, seed=86)
    X = api.PcfSet(o, t * 10.0, v, device=DEV)
    for wname, c in (("exp", 0.0), ("exp", -1.0), ("pow", -1.0), ("pow", math.inf)):
        with pytest.raises(PcfError):
            api.warp(X, wname, c)
    with pytest.raises(PcfError, match="not finite"):  # W(t) = t^301 / 301 overflows
        api.warp(X, "pow", 300.0)
    Xf = api.PcfSet(o, (t * 10.0).astype(np.float32), v.astype(np.float32), device=DEV)
    with pytest.raises(PcfError, match="not finite"):  # beyond FP32's range
        api.warp(Xf, "pow", 40.0)
