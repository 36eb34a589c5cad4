"""Reductions of collections of PCFs (Section 2.1, "Combinations and
reductions"; Section 4, reduction trees and Algorithm ReducePair).

TEST INFRASTRUCTURE ONLY: plain, slow Python written from the paper's
definitions, imported by the tests alone. It shares no code with the GPU
library.

A reduction function h (associative, symmetric) induces f (+) g with
(f (+) g)(t) = h(f(t), g(t)). ReducePair walks the rectangles of the common
refinement of f and g (the distinct breakpoints of either, in increasing
order) and appends (l, h(f(l), g(l))) for a rectangle with left end l when
l = 0 or the value differs from the previous rectangle's. A collection is
reduced by a binary tree: at every level neighbours (2j, 2j+1) are reduced
and an unpaired last item moves up unchanged. From the sum reduction:
mean = (1/n) (+) f_i, and the sample standard deviation
sqrt( (1/(n-1)) (+)_i (f_i - mean)^2 ) (read as 1/(n-1): the printed
normalisation is garbled). A combination of two sets applies ReducePair
with any combination function h (sum, difference, product, max, min,
squared difference) to f_i and g_i. The transformation x -> x/n (or
sqrt(x/(n-1))) is applied to the reduced PCF's values row by row.
"""
from __future__ import annotations

import math

import numpy as np

OPS = {
    "sum": lambda a, b: a + b,
    "max": lambda a, b: a if a >= b else b,
    "min": lambda a, b: a if a <= b else b,
}


def reduce_pair(f, g, h, dtype=np.float64):
    """Algorithm ReducePair: f, g are (t, v) arrays; h a Python function on
    two values of ``dtype``."""
    tf, vf = f
    tg, vg = g
    out_t, out_v = [], []
    i = j = 0  # pieces holding the current rectangle's left end
    v_last = None
    times = sorted(set(tf.tolist()) | set(tg.tolist()))
    for l in times:
        while i + 1 < len(tf) and tf[i + 1] <= l:
            i += 1
        while j + 1 < len(tg) and tg[j + 1] <= l:
            j += 1
        v = dtype(h(dtype(vf[i]), dtype(vg[j])))
        if l == 0 or v != v_last:
            out_t.append(l)
            out_v.append(v)
        v_last = v
    return np.array(out_t, dtype=dtype), np.array(out_v, dtype=dtype)


def tree(items, h, dtype=np.float64):
    """Binary reduction tree over a list of (t, v) PCFs."""
    level = list(items)
    while len(level) > 1:
        nxt = []
        for k in range(0, len(level) - 1, 2):
            nxt.append(reduce_pair(level[k], level[k + 1], h, dtype))
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    return level[0]


def _pieces(offsets, t, v, lo, hi):
    return [(np.asarray(t[offsets[i]:offsets[i + 1]]), np.asarray(v[offsets[i]:offsets[i + 1]]))
            for i in range(lo, hi)]


def reduce_groups(op, groups, offsets, t, v, dtype=np.float64):
    """Reduce each group of PCFs (PCFs groups[b] .. groups[b+1]-1) with
    ``op`` in {"sum", "max", "min", "mean", "std"}. Returns a list of (t, v)."""
    t = np.asarray(t, dtype=dtype)
    v = np.asarray(v, dtype=dtype)
    out = []
    for b in range(len(groups) - 1):
        fs = _pieces(offsets, t, v, groups[b], groups[b + 1])
        n = len(fs)
        if n == 0:
            raise ValueError("empty group")
        if op in OPS:
            out.append(tree(fs, OPS[op], dtype))
            continue
        s_t, s_v = tree(fs, OPS["sum"], dtype)
        mean = (s_t, np.array([x / dtype(n) for x in s_v], dtype=dtype))
        if op == "mean":
            out.append(mean)
            continue
        if op != "std" or n < 2:
            raise ValueError("op must be sum, max, min, mean or std (std needs n >= 2)")
        sq = lambda a, b: (a - b) * (a - b)
        cs = [reduce_pair(f, mean, sq, dtype) for f in fs]
        q_t, q_v = tree(cs, OPS["sum"], dtype)
        out.append((q_t, np.array([math.sqrt(x / dtype(n - 1)) if dtype == np.float64
                                   else np.float32(math.sqrt(np.float32(x / dtype(n - 1))))
                                   for x in q_v], dtype=dtype)))
    return out


COMBINE = dict(OPS, sub=lambda a, b: a - b, mul=lambda a, b: a * b,
               sqdiff=lambda a, b: (a - b) * (a - b))


def combine_sets(op, xs, ys, dtype=np.float64):
    """The induced combination h_*(f_i, g_i) of two sets index by index
    (Section 2.1), each by Algorithm ReducePair; xs and ys are (offsets, t,
    v) triples with the same number of PCFs."""
    (xo, xt, xv), (yo, yt, yv) = xs, ys
    xt, xv = np.asarray(xt, dtype=dtype), np.asarray(xv, dtype=dtype)
    yt, yv = np.asarray(yt, dtype=dtype), np.asarray(yv, dtype=dtype)
    h = COMBINE[op]
    return [reduce_pair((xt[xo[i]:xo[i + 1]], xv[xo[i]:xo[i + 1]]),
                        (yt[yo[i]:yo[i + 1]], yv[yo[i]:yo[i + 1]]), h, dtype)
            for i in range(len(xo) - 1)]


def evaluate(pcf, x):
    """f(x) for a (t, v) PCF at the points x."""
    t, v = pcf
    return v[np.searchsorted(t, x, side="right") - 1]
