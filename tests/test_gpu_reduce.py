"""GPU parity of the reductions (Section 2.1 reductions; Section 4,
Algorithm ReducePair and reduction trees) against the oracle's ReducePair
tree. Both sides pair neighbours level by level and add in the same order,
so FP64 results are compared row for row, bit for bit; FP32 sums, maxima
and minima too, FP32 means and standard deviations pointwise within a few
ulps of the values."""
import numpy as np
import pytest

from oracle import reduce as red
from paper_2404_07183_amd import api, workloads
from paper_2404_07183_amd._lib import PcfError

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
OPS = ["sum", "mean", "max", "min", "std"]


def _rows(S):
    o = S.offsets_host
    t, v = S.t.cpu().numpy(), S.v.cpu().numpy()
    return [(t[o[b]:o[b + 1]], v[o[b]:o[b + 1]]) for b in range(S.n)]


def _tied_set(n, seed, dtype=np.float64):
    """PCFs on a coarse dyadic time grid: many breakpoints shared across PCFs."""
    rng = np.random.default_rng(seed)
    pcfs = []
    for _ in range(n):
        k = int(rng.integers(1, 20))
        ts = np.concatenate([[0.0], np.sort(rng.choice(np.arange(1, 64), k - 1, replace=False))]) / 8
        vs = np.concatenate([rng.standard_normal(k - 1), [0.0]])
        pcfs.append((ts, vs))
    o = np.concatenate([[0], np.cumsum([len(p[0]) for p in pcfs])])
    return (o, np.concatenate([p[0] for p in pcfs]).astype(dtype),
            np.concatenate([p[1] for p in pcfs]).astype(dtype))


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("data", ["uniform", "tied"])
def test_reduce_fp64_bit_exact(op, data):
    if data == "uniform":
        o, t, v = workloads.uniform_counts(120, 1, 60, seed=101)
    else:
        o, t, v = _tied_set(120, seed=102)
    groups = [0, 1, 3, 6, 13, 29, 45, 78, 79, 120] if op != "std" else \
        [0, 2, 5, 12, 29, 45, 78, 80, 120]
    X = api.PcfSet(o, t, v, device=DEV)
    got = _rows(api.reduce(X, op, groups))
    want = red.reduce_groups(op, groups, o, t, v)
    for b, ((gt, gv), (wt, wv)) in enumerate(zip(got, want)):
        assert np.array_equal(gt, wt), (op, b, len(gt), len(wt))
        assert np.array_equal(gv, wv), (op, b)


def test_reduce_deep_tree_and_one_group():
    o, t, v = workloads.uniform_counts(1000, 1, 40, seed=103)
    X = api.PcfSet(o, t, v, device=DEV)
    for op in ("mean", "max"):
        (gt, gv), = _rows(api.reduce(X, op))
        (wt, wv), = red.reduce_groups(op, [0, 1000], o, t, v)
        assert np.array_equal(gt, wt) and np.array_equal(gv, wv), op
    # 250 groups of 4 in one call
    groups = np.arange(0, 1001, 4)
    got = _rows(api.reduce(X, "std", groups))
    want = red.reduce_groups("std", groups, o, t, v)
    assert all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
               for a, b in zip(got, want))


@pytest.mark.parametrize("op", OPS)
def test_reduce_fp32(op):
    o, t, v = workloads.uniform_counts(90, 1, 50, seed=104, dtype=np.float32)
    groups = [0, 2, 9, 40, 90]
    X = api.PcfSet(o, t, v, device=DEV)
    got = _rows(api.reduce(X, op, groups))
    want = red.reduce_groups(op, groups, o, t, v, dtype=np.float32)
    for (gt, gv), (wt, wv) in zip(got, want):
        if op in ("sum", "max", "min"):
            assert np.array_equal(gt, wt) and np.array_equal(gv, wv)
            continue
        x = np.unique(np.concatenate([gt, wt]))
        a = red.evaluate((gt, gv), x).astype(np.float64)
        b = red.evaluate((wt, wv), x).astype(np.float64)
        assert np.all(np.abs(a - b) <= 4 * np.finfo(np.float32).eps * np.abs(b))


def test_reduce_errors():
    o, t, v = workloads.uniform_counts(10, 1, 20, seed=105)
    X = api.PcfSet(o, t, v, device=DEV)
    with pytest.raises(PcfError):
        api.reduce(X, "mean", [0, 4, 4, 10])  # empty group
    with pytest.raises(PcfError):
        api.reduce(X, "std", [0, 1, 10])  # std of one PCF
    with pytest.raises(PcfError):
        api.reduce(X, "mean", [0, 5])  # groups must cover the set


@pytest.mark.parametrize("op", ["sum", "sub", "mul", "max", "min", "sqdiff"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_combine_bit_exact(op, dtype):
    # one arithmetic operation per value on each side, so both precisions
    # agree bit for bit; the tied set shares many breakpoints with itself
    xs = workloads.uniform_counts(150, 1, 80, seed=106, dtype=dtype)
    ys = _tied_set(150, seed=107, dtype=dtype)
    X, Y = api.PcfSet(*xs, device=DEV), api.PcfSet(*ys, device=DEV)
    got = _rows(api.combine(X, Y, op))
    want = red.combine_sets(op, xs, ys, dtype=dtype)
    for i, ((gt, gv), (wt, wv)) in enumerate(zip(got, want)):
        assert np.array_equal(gt, wt) and np.array_equal(gv, wv), (op, i)
    # against itself: f - f is the zero PCF, one row
    Z = _rows(api.combine(X, X, "sub"))
    assert all(len(t) == 1 and t[0] == 0 and v[0] == 0 for t, v in Z)


def test_combine_errors():
    xs = workloads.uniform_counts(10, 1, 20, seed=108)
    X = api.PcfSet(*xs, device=DEV)
    Y = api.PcfSet(*workloads.uniform_counts(11, 1, 20, seed=109), device=DEV)
    with pytest.raises(PcfError):
        api.combine(X, Y, "sum")  # different counts
    Xf = api.PcfSet(xs[0], xs[1].astype(np.float32), xs[2].astype(np.float32), device=DEV)
    with pytest.raises(PcfError):
        api.combine(X, Xf, "sum")  # different dtypes


@pytest.mark.parametrize("data", ["uniform", "tied"])
def test_std_small_and_large_groups_bit_exact(data):
    # groups of up to 64 PCFs take the chunked kernel (PCF rows staged per
    # chunk of root rows), larger ones the per-row search; both in one call,
    # bit for bit against the oracle's tree in FP64
    if data == "uniform":
        o, t, v = workloads.uniform_counts(400, 1, 40, seed=106)
    else:
        o, t, v = _tied_set(400, seed=107)
    groups = [0, 2, 5, 9, 17, 33, 66, 130, 195, 260, 400]  # 2..64, 65, 65, 140
    X = api.PcfSet(o, t, v, device=DEV)
    got = _rows(api.reduce(X, "std", groups))
    want = red.reduce_groups("std", groups, o, t, v)
    for b, ((gt, gv), (wt, wv)) in enumerate(zip(got, want)):
        assert np.array_equal(gt, wt), (data, b, len(gt), len(wt))
        assert np.array_equal(gv, wv), (data, b)


def test_std_group_past_two_to_the_fifteen():
    # one group of 2^15 + 3 PCFs (the second level of the std's subtree
    # counter) next to a small group, bit for bit against the oracle. The
    # PCFs have one or two rows on a grid of eight times, so that the
    # oracle's per-PCF squared deviations stay a few rows long.
    rng = np.random.default_rng(108)
    big = (1 << 15) + 3
    pcfs = []
    for _ in range(big + 5):
        if rng.random() < 0.2:
            pcfs.append((np.array([0.0]), np.array([0.0])))
        else:
            t1 = float(rng.integers(1, 9))
            pcfs.append((np.array([0.0, t1]), np.array([float(rng.integers(-8, 9)) / 4, 0.0])))
    o = np.concatenate([[0], np.cumsum([len(p[0]) for p in pcfs])]).astype(np.int64)
    t = np.concatenate([p[0] for p in pcfs])
    v = np.concatenate([p[1] for p in pcfs])
    groups = [0, 5, 5 + big]
    X = api.PcfSet(o, t, v, device=DEV)
    got = _rows(api.reduce(X, "std", groups))
    want = red.reduce_groups("std", groups, o, t, v)
    for b, ((gt, gv), (wt, wv)) in enumerate(zip(got, want)):
        assert np.array_equal(gt, wt), (b, gt, wt)
        assert np.array_equal(gv, wv), (b, gv, wv)


def test_std_tie_runs_across_chunk_edges():
    # PCFs of a group that share every breakpoint: the root holds runs of m
    # equal times, and the 1,024-row chunk edges of the standard deviation's
    # root pass fall inside them (1024 is not a multiple of 60 or 63). This is
    # the largest window of PCF rows a chunk can select; bit for bit against
    # the oracle.
    rng = np.random.default_rng(109)
    pcfs = []
    for m, k in ((60, 50), (63, 40), (2, 700), (64, 17)):
        ts = np.arange(k, dtype=np.float64) / 4
        for _ in range(m):
            vs = np.concatenate([rng.integers(-16, 17, size=k - 1) / 8, [0.0]])
            pcfs.append((ts, vs))
    o = np.concatenate([[0], np.cumsum([len(p[0]) for p in pcfs])]).astype(np.int64)
    t = np.concatenate([p[0] for p in pcfs])
    v = np.concatenate([p[1] for p in pcfs])
    groups = [0, 60, 123, 125, 189]
    X = api.PcfSet(o, t, v, device=DEV)
    got = _rows(api.reduce(X, "std", groups))
    want = red.reduce_groups("std", groups, o, t, v)
    for b, ((gt, gv), (wt, wv)) in enumerate(zip(got, want)):
        assert np.array_equal(gt, wt), (b, len(gt), len(wt))
        assert np.array_equal(gv, wv), b


def test_std_full_size_groups_of_twenty():
    # the 20,000-PCF set (counts 50..500) in 1,000 groups of 20, as timed;
    # five groups (the first, the last and three drawn at random) bit for bit
    # against the oracle run on those groups alone
    o, t, v = workloads.config_plain()
    groups = np.arange(0, len(o), 20)
    X = api.PcfSet(o, t, v, device=DEV)
    got = _rows(api.reduce(X, "std", groups))
    rng = np.random.default_rng(110)
    for b in [0, len(groups) - 2] + list(rng.integers(1, len(groups) - 2, size=3)):
        i0, i1 = groups[b], groups[b + 1]
        so = o[i0:i1 + 1] - o[i0]
        want = red.reduce_groups("std", [0, i1 - i0], so, t[o[i0]:o[i1]], v[o[i0]:o[i1]])
        assert np.array_equal(got[b][0], want[0][0]), b
        assert np.array_equal(got[b][1], want[0][1]), b
