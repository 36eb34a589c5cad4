"""GPU parity of the integrals over a range [a, b) (Section 2.2): the
restriction transform against a NumPy restriction (bit for bit), and the
matrices of restricted sets against the oracle's bounded integrals.

Bars: FP64 |gpu - oracle| <= 1e-12 * scale; FP32 against the oracle on the
rounded inputs and bounds at 1e-5 * scale.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2404_07183_amd import api, workloads
from paper_2404_07183_amd._lib import PcfError
from test_oracle_bounds import restrict as np_restrict

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
INF = math.inf
BOUNDS = [(0.0, INF), (0.0, 25.0), (3.5, 60.0), (20.0, INF), (0.25, 0.75)]

KINDS = {  # name -> (api call with bounds, oracle kind, p)
    "l1": (lambda X, b: api.pdist(X, 1.0, bounds=b), oracle.LP, 1.0),
    "l2": (lambda X, b: api.pdist(X, 2.0, bounds=b), oracle.LP, 2.0),
    "gram": (lambda X, b: api.gram(X, bounds=b), oracle.GRAM, 0.0),
    "l3.5pow": (lambda X, b: api.pdist(X, 3.5, power=True, bounds=b), oracle.LP_POW, 3.5),
}


def test_restriction_matches_numpy():
    o, t, v = workloads.uniform_counts(300, 1, 90, seed=61)
    X = api.PcfSet(o, t, v, device=DEV)
    for a, b in BOUNDS + [(5.0, 5.5)]:
        R = api.restrict(X, a, b)
        ro, rt, rv = R.offsets_host, R.t.cpu().numpy(), R.v.cpu().numpy()
        for i in range(X.n):
            et, ev = np_restrict(t[o[i]:o[i + 1]], v[o[i]:o[i + 1]], a, b)
            assert np.array_equal(rt[ro[i]:ro[i + 1]], et), (a, b, i)
            assert np.array_equal(rv[ro[i]:ro[i + 1]], ev), (a, b, i)


@pytest.mark.parametrize("name", sorted(KINDS))
def test_bounded_matrices_fp64(name):
    fn, okind, p = KINDS[name]
    o, t, v = workloads.uniform_counts(120, 1, 150, seed=62)
    X = api.PcfSet(o, t, v, device=DEV)
    n = X.n
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for bnd in BOUNDS:
        M = fn(X, bnd).cpu().numpy()
        ref, ab = oracle.entries_ab(okind, p, bnd[0], bnd[1], o, t, v, I.ravel(), J.ravel(),
                                    with_abs=True)
        sc = ab if (okind != oracle.LP or p == 1.0) else ab ** (1.0 / p)
        err = np.abs(M.ravel() - ref)
        bad = err > 1e-12 * np.maximum(sc, 1e-300)
        assert not bad.any(), (name, bnd, np.argwhere(bad)[:5], err[bad][:5])


def test_bounded_fp32_and_cross():
    o, t, v = workloads.uniform_counts(150, 10, 200, seed=63, dtype=np.float32)
    X = api.PcfSet(o, t, v, device=DEV)
    a, b = 2.1, 47.3
    fa, fb = float(np.float32(a)), float(np.float32(b))
    M = api.pdist(X, 1.0, bounds=(a, b)).cpu().numpy().astype(np.float64)
    I, J = np.meshgrid(np.arange(X.n), np.arange(X.n), indexing="ij")
    ref, ab = oracle.entries_ab(oracle.LP, 1.0, fa, fb, o, t, v, I.ravel(), J.ravel(),
                                with_abs=True)
    assert np.all(np.abs(M.ravel() - ref) <= 1e-5 * np.maximum(ab, 1e-300))
    # cross-set with bounds: the X x Y block of the bounded joint matrix
    ys = workloads.uniform_counts(40, 10, 200, seed=64, dtype=np.float32)
    Y = api.PcfSet(*ys, device=DEV)
    C = api.cross_gram(X, Y, bounds=(a, b)).cpu().numpy().astype(np.float64)
    oj = np.concatenate([o, o[-1] + ys[0][1:]])
    tj, vj = np.concatenate([t, ys[1]]), np.concatenate([v, ys[2]])
    Ic, Jc = np.meshgrid(np.arange(X.n), X.n + np.arange(Y.n), indexing="ij")
    refc, abc = oracle.entries_ab(oracle.GRAM, 0.0, fa, fb, oj, tj, vj, Ic.ravel(),
                                  Jc.ravel(), with_abs=True)
    assert np.all(np.abs(C.ravel() - refc) <= 1e-5 * np.maximum(abc, 1e-300))


def test_bounds_errors():
    o, t, v = workloads.uniform_counts(10, 1, 20, seed=65)
    X = api.PcfSet(o, t, v, device=DEV)
    for a, b in ((2.0, 2.0), (-1.0, 3.0), (3.0, 1.0), (INF, INF)):
        with pytest.raises(PcfError):
            api.restrict(X, a, b)
    Xf = api.PcfSet(o, t.astype(np.float32), v.astype(np.float32), device=DEV)
    with pytest.raises(PcfError):  # ordered in FP64, equal in FP32
        api.restrict(Xf, 1.0, 1.0 + 1e-12)
