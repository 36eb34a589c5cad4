"""GPU parity of the single-PCF functionals (Section 3.2: integrals, L_p
norms and the sup norm over [a, b)) against the oracle's segment iteration.

Bars: FP64 |gpu - oracle| <= 1e-12 * scale (scale = sum |h| * width, its
p-th root for a norm), FP32 against the oracle on the rounded inputs at
1e-5 * scale.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2404_07183_amd import api, workloads
from paper_2404_07183_amd._lib import PcfError

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
INF = math.inf

CASES = [  # name, api call, oracle kind, p
    ("integral", lambda X, a, b: api.integrals(X, a, b), oracle.S_INTEGRAL, 1.0),
    ("norm1", lambda X, a, b: api.norms(X, 1.0, a, b), oracle.S_NORM, 1.0),
    ("norm2", lambda X, a, b: api.norms(X, 2.0, a, b), oracle.S_NORM, 2.0),
    ("norm2pow", lambda X, a, b: api.norms(X, 2.0, a, b, power=True), oracle.S_NORM_POW, 2.0),
    ("norm3.5", lambda X, a, b: api.norms(X, 3.5, a, b), oracle.S_NORM, 3.5),
    ("norminf", lambda X, a, b: api.norms(X, INF, a, b), oracle.S_NORM_INF, 0.0),
]
BOUNDS = [(0.0, INF), (0.0, 7.5), (3.25, 40.0), (12.0, INF), (500.0, INF)]


def _check(o, t, v, dtype, tol):
    X = api.PcfSet(o, t.astype(dtype), v.astype(dtype), device=DEV)
    t64, v64 = t.astype(dtype).astype(np.float64), v.astype(dtype).astype(np.float64)
    for name, fn, kind, p in CASES:
        for a, b in BOUNDS:
            got = fn(X, a, b).cpu().numpy().astype(np.float64)
            ref, ab = oracle.single(kind, p, a, b, o, t64, v64, with_abs=True)
            sc = ab if (kind != oracle.S_NORM or p == 1.0) else ab ** (1.0 / p)
            err = np.abs(got - ref)
            bad = err > tol * np.maximum(sc, 1e-300)
            assert not bad.any(), (name, a, b, np.argwhere(bad)[:5], err[bad][:5])


def test_single_fp64():
    # short and long PCFs (several waves' worth of rows), lengths 1..700
    o, t, v = workloads.uniform_counts(500, 1, 700, seed=51)
    _check(o, t, v, np.float64, 1e-12)


def test_single_fp32():
    o, t, v = workloads.uniform_counts(300, 1, 400, seed=52)
    _check(o, t, v, np.float32, 1e-5)


def test_single_round_boundaries():
    # a lane loads four 64-row rounds before adding: PCFs whose row counts
    # sit on either side of 64, 128, 256 and 512 rows, in mixed order
    counts = np.array([1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513,
                       1000] * 3)
    rng = np.random.default_rng(54)
    counts = counts[rng.permutation(len(counts))]
    P = int(counts.sum())
    o, t, v = workloads._assemble(counts, rng.exponential(1.0, P), rng.standard_normal(P))
    _check(o, t, v, np.float64, 1e-12)
    _check(*workloads.to_dtype(o, t, v, np.float32), np.float32, 1e-5)


def test_single_more_pcfs_than_waves():
    # 40,000 PCFs: more than the launch's 32,768 waves, so waves take a
    # second PCF (whose offsets were loaded while the first was summed)
    o, t, v = workloads.uniform_counts(40000, 1, 12, seed=55)
    _check(o, t, v, np.float64, 1e-12)


def test_single_full_size_against_pairwise():
    # on the plain 20,000-PCF set: int f^2 equals the Gram diagonal computed
    # by the pairwise kernel, and the norms match the oracle on a sample
    o, t, v = workloads.config_plain()
    X = api.PcfSet(o, t, v, device=DEV)
    n2 = api.norms(X, 2.0, power=True).cpu().numpy()
    Y = api.PcfSet(o[:2001], t[:o[2000]], v[:o[2000]], device=DEV)
    G = api.gram(Y).cpu().numpy()
    assert np.allclose(n2[:2000], np.diag(G), rtol=1e-12, atol=0)
    idx = np.random.default_rng(53).integers(0, X.n, 500)
    ref, ab = oracle.single(oracle.S_NORM_POW, 2.0, 0.0, INF, o, t, v, with_abs=True)
    assert np.all(np.abs(n2[idx] - ref[idx]) <= 1e-12 * ab[idx])


def test_single_tail_and_errors():
    o = np.array([0, 2, 3])
    t = np.array([0.0, 1.5, 0.0])
    v = np.array([2.0, -1.0, 0.0])  # PCF 0 ends at -1: infinite over [0, inf)
    X = api.PcfSet(o, t, v, device=DEV)
    I = api.integrals(X).cpu().numpy()
    assert I[0] == -INF and I[1] == 0.0
    assert api.norms(X, 1.0).cpu().numpy()[0] == INF
    assert api.integrals(X, 0.0, 3.0).cpu().numpy()[0] == 2.0 * 1.5 - 1.5
    for a, b in ((1.0, 1.0), (-1.0, 2.0), (2.0, 1.0)):
        with pytest.raises(PcfError):
            api.integrals(X, a, b)
    with pytest.raises(PcfError):
        api.norms(X, 0.5)
