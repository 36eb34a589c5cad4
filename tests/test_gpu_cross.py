"""GPU parity of the cross-set matrix (two collections, X rows x Y columns)
against the oracle on one CSR of X then Y (the same integrals).

Bars as for the single-set matrix: FP64 |gpu - oracle| <= 1e-12 * scale,
FP32 against the oracle on the rounded inputs at 1e-5 * scale.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2404_07183_amd import api, workloads
from paper_2404_07183_amd._lib import PcfError

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

KINDS = {  # name -> (api call, oracle kind, p)
    "l1": (lambda X, Y, **k: api.cdist(X, Y, 1.0, **k), oracle.LP, 1.0),
    "l2": (lambda X, Y, **k: api.cdist(X, Y, 2.0, **k), oracle.LP, 2.0),
    "l2sq": (lambda X, Y, **k: api.cdist(X, Y, 2.0, power=True, **k), oracle.LP_POW, 2.0),
    "gram": (lambda X, Y, **k: api.cross_gram(X, Y, **k), oracle.GRAM, 0.0),
    "l3.5": (lambda X, Y, **k: api.cdist(X, Y, 3.5, **k), oracle.LP, 3.5),
}


def _concat(a, b):
    (oa, ta, va), (ob, tb, vb) = a, b
    o = np.concatenate([oa, oa[-1] + ob[1:]])
    return o, np.concatenate([ta, tb]), np.concatenate([va, vb])


def _check(name, xs, ys, tol):
    fn, okind, p = KINDS[name]
    X = api.PcfSet(*xs, device=DEV)
    Y = api.PcfSet(*ys, device=DEV)
    M = fn(X, Y).cpu().numpy().astype(np.float64)
    nx, ny = len(xs[0]) - 1, len(ys[0]) - 1
    assert M.shape == (nx, ny)
    o, t, v = _concat(xs, ys)
    I, J = np.meshgrid(np.arange(nx), nx + np.arange(ny), indexing="ij")
    ref, ab = oracle.entries(okind, p, o, t.astype(np.float64), v.astype(np.float64),
                             I.ravel(), J.ravel(), with_abs=True)
    ref = ref.reshape(M.shape)
    sc = ab.reshape(M.shape)
    if okind == oracle.LP and p != 1.0:
        sc = sc ** (1.0 / p)
    err = np.abs(M - ref)
    bad = err > tol * np.maximum(sc, 1e-300)
    assert not bad.any(), (name, np.argwhere(bad)[:5], err[bad][:5])


@pytest.mark.parametrize("name", sorted(KINDS))
def test_cross_fp64(name):
    xs = workloads.uniform_counts(150, 5, 400, seed=31)
    ys = workloads.uniform_counts(230, 1, 120, seed=32)
    _check(name, xs, ys, 1e-12)


@pytest.mark.parametrize("name", ["l1", "gram"])
def test_cross_fp32(name):
    xs = workloads.uniform_counts(200, 50, 500, seed=33, dtype=np.float32)
    ys = workloads.uniform_counts(90, 10, 300, seed=34, dtype=np.float32)
    _check(name, xs, ys, 1e-5)


def test_cross_equals_window_of_the_joint_set():
    # X x Y is the off-diagonal window of the matrix of X then Y
    xs = workloads.uniform_counts(120, 20, 200, seed=35)
    ys = workloads.uniform_counts(70, 20, 200, seed=36)
    o, t, v = _concat(xs, ys)
    Z = api.PcfSet(o, t, v, device=DEV)
    W = api.pdist(Z, 1.0, window=(0, 120, 120, 190)).cpu().numpy()
    C = api.cdist(api.PcfSet(*xs, device=DEV), api.PcfSet(*ys, device=DEV)).cpu().numpy()
    assert np.allclose(C, W, rtol=1e-13, atol=0)


def test_cross_edges_and_errors():
    xs = workloads.uniform_counts(5, 1, 4, seed=37)
    ys = workloads.uniform_counts(3, 1, 4, seed=38)
    X, Y = api.PcfSet(*xs, device=DEV), api.PcfSet(*ys, device=DEV)
    E = api.PcfSet(np.array([0]), np.zeros(0), np.zeros(0), device=DEV)
    assert api.cdist(X, E).shape == (5, 0) and api.cdist(E, Y).shape == (0, 3)
    # self-distances of X against a copy of X: zero diagonal
    D = api.cdist(X, api.PcfSet(*xs, device=DEV)).cpu().numpy()
    assert np.all(np.diag(D) == 0)
    with pytest.raises(ValueError):
        api.cdist(X, api.PcfSet(ys[0], ys[1].astype(np.float32), ys[2].astype(np.float32),
                                device=DEV))
    # a contract violation in Y is reported under PCF_VALIDATE
    o, t, v = ys
    v = v.copy()
    v[o[2] - 1] = 1.0  # PCF 1 of Y does not end at 0
    with pytest.raises(PcfError, match="Y PCF 1"):
        api.cdist(X, api.PcfSet(o, t, v, device=DEV), validate=True)
