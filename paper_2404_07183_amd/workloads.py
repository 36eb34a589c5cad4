"""Seeded synthetic PCF workloads (inputs only; no integral arithmetic here).

Every generator returns host NumPy CSR arrays ``(offsets, t, v)``: PCF ``i``
owns rows ``offsets[i] .. offsets[i+1]-1`` of ``t`` (breakpoint times) and
``v`` (values). The shared recipe (a PCF of ``n`` rows):

* ``t_0 = 0`` and ``t_k = t_{k-1} + Exp(1)`` for ``k = 1..n-1``;
* ``v_k ~ N(0, 1)`` for ``k <= n-2`` and ``v_{n-1} = 0`` (eventually zero,
  so integrals over ``[0, inf)`` are finite -- the paper's Appendix A also ends
  every synthetic PCF at value 0);
* FP32 data are the FP64 draws rounded to nearest; a time that rounds onto
  its predecessor drops the earlier row (the later row wins), which keeps
  times strictly increasing.

Draw order is fixed (counts, then gaps, then values) so a seed names one
dataset. These shapes stand in for the paper's synthetic benchmark data
(Appendix A: counts 10..1000, several time scales); the paper uses no public
dataset.
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def _assemble(counts, gaps, values):
    """CSR arrays from per-PCF counts, a flat array of gaps (the entry at each
    PCF start is ignored) and a flat array of values (the last one of each PCF
    is overwritten with 0)."""
    counts = np.asarray(counts, dtype=np.int64)
    offsets = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    P = int(offsets[-1])
    t = np.empty(P, dtype=np.float64)
    for i in range(len(counts)):
        a, b = offsets[i], offsets[i + 1]
        if b - a == 0:
            continue
        seg = gaps[a:b].copy()
        seg[0] = 0.0
        np.cumsum(seg, out=t[a:b])
    v = np.array(values[:P], dtype=np.float64, copy=True)
    v[offsets[1:] - 1] = 0.0
    return dedup(offsets, t, v)


def dedup(offsets, t, v):
    """Drop rows whose time equals the previous row's time inside the same
    PCF (the later row is kept). Returns new ``(offsets, t, v)``."""
    offsets = np.asarray(offsets, dtype=np.int64)
    P = len(t)
    if P == 0:
        return offsets.copy(), t.copy(), v.copy()
    starts = np.zeros(P, dtype=bool)
    starts[offsets[:-1][offsets[:-1] < offsets[1:]]] = True
    # row k is dropped when row k+1 has the same time and is in the same PCF
    same_next = np.zeros(P, dtype=bool)
    same_next[:-1] = (t[1:] == t[:-1]) & ~starts[1:]
    keep = ~same_next
    if keep.all():
        return offsets.copy(), t.copy(), v.copy()
    pcf_of_row = np.repeat(np.arange(len(offsets) - 1), np.diff(offsets))
    new_counts = np.bincount(pcf_of_row[keep], minlength=len(offsets) - 1)
    new_off = np.zeros(len(offsets), dtype=np.int64)
    np.cumsum(new_counts, out=new_off[1:])
    t2, v2 = t[keep].copy(), v[keep].copy()
    # a PCF whose first row was dropped now starts at the later row, whose
    # time is also 0 (equal times), so t_0 = 0 still holds
    return new_off, t2, v2


def to_dtype(offsets, t, v, dtype):
    """Round to ``dtype`` (float32 or float64), then remove duplicate times."""
    dtype = np.dtype(dtype)
    if dtype == np.float64:
        return offsets, t, v
    t32 = t.astype(dtype)
    v32 = v.astype(dtype)
    o, t2, v2 = dedup(offsets, t32, v32)
    return o, t2, v2


def uniform_counts(N, nmin, nmax, seed, dtype=np.float64):
    """N PCFs, row counts uniform on {nmin..nmax}, Exp(1) gaps, N(0,1) values,
    last value 0."""
    rng = _rng(seed)
    counts = rng.integers(nmin, nmax + 1, size=N)
    P = int(counts.sum())
    gaps = rng.exponential(1.0, size=P)
    values = rng.standard_normal(size=P)
    o, t, v = _assemble(counts, gaps, values)
    return to_dtype(o, t, v, dtype)


def config_plain_small(seed=1):
    """N = 200 PCFs, counts U{10..100}, FP64 (plain L1 matrix, small case)."""
    return uniform_counts(200, 10, 100, seed)


def config_plain(seed=2, dtype=np.float64, N=20000):
    """N = 20,000 PCFs, counts U{50..500} (L1, L2, Gram; FP32 and FP64)."""
    return uniform_counts(N, 50, 500, seed, dtype)


def config_batched(seed=3, B=512, smin=16, smax=2048, mean_len=200,
                   cap=5000):
    """B independent problems: set sizes round(exp(U(ln smin, ln smax))),
    per-PCF counts Geometric(p = 1/mean_len) on {1, 2, ...} capped at
    ``cap`` (a count of 1 is the zero PCF). FP64.

    Returns ``(set_offsets, offsets, t, v)``; problem ``b`` owns PCFs
    ``set_offsets[b] .. set_offsets[b+1]-1`` of the one CSR set."""
    rng = _rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(smin), math.log(smax),
                                       size=B))).astype(np.int64)
    M = int(sizes.sum())
    counts = np.minimum(rng.geometric(1.0 / mean_len, size=M), cap)
    P = int(counts.sum())
    gaps = rng.exponential(1.0, size=P)
    values = rng.standard_normal(size=P)
    o, t, v = _assemble(counts, gaps, values)
    set_offsets = np.zeros(B + 1, dtype=np.int64)
    np.cumsum(sizes, out=set_offsets[1:])
    return set_offsets, o, t, v


def config_grad(seed=4, N=4096):
    """N = 4,096 PCFs, counts U{20..300}, FP64, plus the loss weights W, U:
    upper triangle (diagonal included) i.i.d. U(0,1), mirrored.

    Returns ``(offsets, t, v, W, U)``."""
    o, t, v = uniform_counts(N, 20, 300, seed)
    rng = _rng(seed + 1000)
    W = np.triu(rng.uniform(0.0, 1.0, size=(N, N)))
    W = W + np.triu(W, 1).T
    U = np.triu(rng.uniform(0.0, 1.0, size=(N, N)))
    U = U + np.triu(U, 1).T
    return o, t, v, W, U


def stable_rank_like(N, nmin, nmax, seed, dtype=np.float32, lam=50.0):
    """Nonincreasing, nonnegative integer-valued PCFs: counts U{nmin..nmax},
    Exp(1) gaps, v_0 ~ Poisson(lam), then v_k = floor((1 - S_k / S_n) *
    (v_0 + 1)) capped at v_0, with S_k partial sums of Exp(1) draws (sorted
    uniforms, descending), and v_{n-1} = 0. Many consecutive equal values, i.e.
    discretizations that are not minimal."""
    rng = _rng(seed)
    counts = rng.integers(nmin, nmax + 1, size=N)
    P = int(counts.sum())
    gaps = rng.exponential(1.0, size=P)
    v0 = rng.poisson(lam, size=N).astype(np.float64)
    e = rng.exponential(1.0, size=P)
    offsets = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    cs = np.cumsum(e)
    seg_before = np.concatenate([[0.0], cs[offsets[1:-1] - 1]])
    pcf = np.repeat(np.arange(N), counts)
    S = cs - seg_before[pcf]
    T = S[offsets[1:] - 1][pcf]
    vals = np.minimum(np.floor((1.0 - S / T) * (v0[pcf] + 1.0)), v0[pcf])
    vals[offsets[:-1]] = v0
    del cs, S, T, pcf, e
    o, t, v = _assemble(counts, gaps, vals)
    return to_dtype(o, t, v, dtype)


def config_strip(seed=5, N=500000):
    """The 500,000-PCF stress set: stable-rank-like PCFs, counts U{100..1000},
    FP32. One GPU's share is the 62,500 x 500,000 strip of its L1 matrix."""
    return stable_rank_like(N, 100, 1000, seed, np.float32)


def appendix_shaped(N, seed, dtype=np.float64):
    """PCFs shaped like the paper's Appendix A generator: n ~ U{10..1000},
    a scale alpha ~ N(0,1) per PCF, n-1 times |alpha| * sorted |N(0,1)| draws
    after t_0 = 0 (magnitudes keep the times nonnegative), values N(0,1) and a
    final 0."""
    rng = _rng(seed)
    counts = rng.integers(10, 1001, size=N)
    alpha = np.abs(rng.standard_normal(size=N))
    P = int(counts.sum())
    raw = np.abs(rng.standard_normal(size=P))
    values = rng.standard_normal(size=P)
    offsets = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    t = np.empty(P, dtype=np.float64)
    for i in range(N):
        a, b = offsets[i], offsets[i + 1]
        t[a] = 0.0
        t[a + 1:b] = np.sort(raw[a + 1:b]) * alpha[i]
    v = values.copy()
    v[offsets[1:] - 1] = 0.0
    # equal or zero times after scaling are removed like FP32 duplicates
    o, t, v = dedup(offsets, t, v)
    return to_dtype(o, t, v, dtype)


def random_pairs(N, count, seed, upper=True):
    """``count`` random (i, j) index pairs, i < j when ``upper``."""
    rng = _rng(seed)
    i = rng.integers(0, N, size=count)
    j = rng.integers(0, N, size=count)
    if upper:
        lo, hi = np.minimum(i, j), np.maximum(i, j)
        hi = np.where(lo == hi, np.minimum(hi + 1, N - 1), hi)
        lo = np.where(lo == hi, np.maximum(lo - 1, 0), lo)
        return lo, hi
    return i, j
