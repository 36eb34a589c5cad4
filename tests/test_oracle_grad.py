"""Pins of the oracle's adjoint (not in the paper; reading in oracle/pcf_oracle.c).

* central finite differences of the forward oracle (an independent route to
  the same derivative),
* Euler's identity for homogeneous functions: I is homogeneous of degree 1 in
  the times (t_0 = 0 fixed) and of degree q in the values (q = 2 for d_2^2 and
  the inner product, q = p for d_p^p),
* linearity of the Gram loss: dL/dv_i[k] = integral over piece k of
  sum_j (G_ij + G_ji) f_j, evaluated by dense resampling.
These inputs are tie-free (continuous random times), where the one-sided
time derivatives agree. At a breakpoint shared by two different PCFs the
oracle takes the mean of the one-sided derivatives; that convention is pinned
by exact one-sided differences of the forward oracle on dyadic data
(test_tie_averaged_time_derivative).
"""
import numpy as np
import pytest

import oracle


def _rand_set(rng, M, nmin=2, nmax=12):
    counts = rng.integers(nmin, nmax + 1, size=M)
    off = np.zeros(M + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    t = np.empty(off[-1])
    v = rng.standard_normal(off[-1])
    for i in range(M):
        a, b = off[i], off[i + 1]
        t[a] = 0.0
        t[a + 1:b] = np.cumsum(rng.uniform(0.3, 1.7, size=b - a - 1))
        v[b - 1] = 0.0
    return off, t, v


def _loss(kind, p, off, t, v, G):
    return float(np.sum(G * oracle.matrix(kind, p, off, t, v)))


@pytest.mark.parametrize("kind,p", [(oracle.LP, 1.0), (oracle.LP, 2.0),
                                    (oracle.LP_POW, 2.0), (oracle.GRAM, 0.0),
                                    (oracle.LP, 3.0)])
def test_finite_differences(kind, p):
    rng = np.random.default_rng(11 + int(p * 10) + kind)
    M = 5
    off, t, v = _rand_set(rng, M)
    G = rng.uniform(0, 1, size=(M, M))
    gt, gv = oracle.backward(kind, p, off, t, v, G)
    h = 1e-6
    first = off[:-1]
    last = off[1:] - 1
    for k in range(len(t)):
        if k in set(first.tolist()):
            assert gt[k] == 0.0
        else:
            tp, tm = t.copy(), t.copy()
            tp[k] += h
            tm[k] -= h
            fd = (_loss(kind, p, off, tp, v, G) - _loss(kind, p, off, tm, v, G)) / (2 * h)
            assert gt[k] == pytest.approx(fd, rel=1e-6, abs=1e-7), ("t", k)
        if k in set(last.tolist()):
            assert gv[k] == 0.0
        else:
            vp, vm = v.copy(), v.copy()
            vp[k] += h
            vm[k] -= h
            fd = (_loss(kind, p, off, t, vp, G) - _loss(kind, p, off, t, vm, G)) / (2 * h)
            assert gv[k] == pytest.approx(fd, rel=1e-6, abs=1e-7), ("v", k)


@pytest.mark.parametrize("kind,p,deg", [(oracle.LP_POW, 2.0, 2.0), (oracle.GRAM, 0.0, 2.0),
                                        (oracle.LP_POW, 1.0, 1.0), (oracle.LP_POW, 3.0, 3.0)])
def test_euler_homogeneity(kind, p, deg):
    """sum_k t_k dL/dt_k = L and sum_k v_k dL/dv_k = deg * L (last values are
    0 and t_0 = 0, so the fixed parameters drop out of both sums)."""
    rng = np.random.default_rng(21 + kind)
    M = 6
    off, t, v = _rand_set(rng, M, nmax=20)
    G = rng.uniform(0, 1, size=(M, M))
    L = _loss(kind, p, off, t, v, G)
    gt, gv = oracle.backward(kind, p, off, t, v, G)
    assert float(np.dot(t, gt)) == pytest.approx(L, rel=1e-11)
    assert float(np.dot(v, gv)) == pytest.approx(deg * L, rel=1e-11)


def test_gram_linearity_dense():
    """dL/dv_i[k] for L = sum_ij G_ij <f_i, f_j> is the integral over piece k
    of f_i of sum_j (G_ij + G_ji) f_j. Dyadic times on a 1/4 grid make a
    midpoint resampling of that integral exact."""
    rng = np.random.default_rng(31)
    M = 4
    pcfs = []
    for _ in range(M):
        n = int(rng.integers(2, 8))
        ticks = np.sort(rng.choice(np.arange(1, 40), size=n - 1, replace=False)) / 4.0
        tt = np.concatenate([[0.0], ticks])
        vv = rng.integers(-6, 7, size=n) / 2.0
        vv[-1] = 0.0
        pcfs.append((tt, vv))
    off = np.zeros(M + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(a) for a, _ in pcfs])
    t = np.concatenate([a for a, _ in pcfs])
    v = np.concatenate([b for _, b in pcfs])
    G = rng.integers(0, 5, size=(M, M)).astype(float)
    gt, gv = oracle.backward(oracle.GRAM, 0.0, off, t, v, G)
    T = max(a[-1] for a, _ in pcfs)
    mids = (np.arange(int(T * 4)) + 0.5) / 4.0
    vals = np.stack([b[np.searchsorted(a, mids, side="right") - 1] for a, b in pcfs])
    S = (G + G.T) @ vals  # sum_j (G_ij + G_ji) f_j at each midpoint
    for i, (a, b) in enumerate(pcfs):
        piece = np.searchsorted(a, mids, side="right") - 1
        for k in range(len(a) - 1):
            exp = float(np.sum(S[i][piece == k]) * 0.25)
            assert gv[off[i] + k] == exp


def _dyadic_tied_set(rng, M=6, grid=8, span=3):
    """PCFs whose interior breakpoints sit on the grid k/grid, so that
    breakpoints of different PCFs coincide; dyadic values."""
    counts = rng.integers(4, 10, size=M)
    off = np.zeros(M + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    t = np.empty(off[-1])
    v = np.empty(off[-1])
    for i in range(M):
        a, b = off[i], off[i + 1]
        n = b - a
        t[a] = 0.0
        t[a + 1:b] = np.sort(rng.choice(np.arange(1, span * grid), n - 1, replace=False)) / grid
        v[a:b - 1] = rng.integers(-32, 33, size=n - 1) / 8.0
        v[b - 1] = 0.0
    return off, t, v


@pytest.mark.parametrize("kind,p", [(oracle.LP, 1.0), (oracle.LP_POW, 2.0),
                                    (oracle.GRAM, 0.0), (oracle.LP_POW, 3.0)])
def test_tie_averaged_time_derivative(kind, p):
    """At a breakpoint shared by two different PCFs the loss has a kink in
    that time; the oracle's reading is the mean of the one-sided derivatives.
    Both one-sided derivatives are taken here from the forward oracle by
    one-sided differences: with dyadic times, values and weights and a step
    h = 1/64 (below the grid spacing 1/8, so no breakpoint is crossed) every
    integral is exact and the loss is linear on each side of the kink, so the
    difference quotients are the exact one-sided derivatives."""
    rng = np.random.default_rng(31 + kind + int(p))
    off, t, v = _dyadic_tied_set(rng)
    M = len(off) - 1
    G = rng.integers(0, 17, size=(M, M)) / 16.0
    gt, _ = oracle.backward(kind, p, off, t, v, G)
    h = 1.0 / 64
    L0 = _loss(kind, p, off, t, v, G)
    first = set(off[:-1].tolist())
    owner = np.repeat(np.arange(M), np.diff(off))
    kinks = 0
    for k in range(len(t)):
        if k in first:
            continue
        tp, tm = t.copy(), t.copy()
        tp[k] += h
        tm[k] -= h
        right = (_loss(kind, p, off, tp, v, G) - L0) / h
        left = (L0 - _loss(kind, p, off, tm, v, G)) / h
        tied = np.any((t == t[k]) & (owner != owner[k]))
        if not tied:
            assert right == pytest.approx(left, rel=1e-12, abs=1e-12)
        elif right != left:
            kinks += 1
        assert gt[k] == pytest.approx(0.5 * (right + left), rel=1e-12, abs=1e-12), k
    # the set really exercises the convention: several tied breakpoints
    # whose one-sided derivatives differ
    assert kinks >= 3
