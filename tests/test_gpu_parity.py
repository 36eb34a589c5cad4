"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bars: FP64 |gpu - oracle| <= 1e-12 * scale per entry, where scale is
sum |h| * width of the entry (for d_p: that sum to the power 1/p; for
distances it equals the result). FP32 inputs are compared with the oracle run
on the FP32-rounded inputs at 1e-5 * scale. Dyadic inputs (every width,
product and partial sum exact) must match bit for bit, and every symmetric
output must be bitwise symmetric.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2404_07183_amd import api, workloads

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
DEV = "cuda:0"

KINDS = {  # name -> (api call, oracle kind, p)
    "l1": (lambda X, **k: api.pdist(X, 1.0, **k), oracle.LP, 1.0),
    "l2": (lambda X, **k: api.pdist(X, 2.0, **k), oracle.LP, 2.0),
    "l2sq": (lambda X, **k: api.pdist(X, 2.0, power=True, **k), oracle.LP_POW, 2.0),
    "gram": (lambda X, **k: api.gram(X, **k), oracle.GRAM, 0.0),
    "l3.5": (lambda X, **k: api.pdist(X, 3.5, **k), oracle.LP, 3.5),  # products and sqrt
    "l3pow": (lambda X, **k: api.pdist(X, 3.0, power=True, **k), oracle.LP_POW, 3.0),
    "l1.5": (lambda X, **k: api.pdist(X, 1.5, **k), oracle.LP, 1.5),
    "l2.7": (lambda X, **k: api.pdist(X, 2.7, **k), oracle.LP, 2.7),  # pow
}


def _scale(okind, p, ab):
    if okind == oracle.LP and p != 1.0:
        return ab ** (1.0 / p)
    return ab


def _check_full(name, o, t, v, tol, window=None):
    fn, okind, p = KINDS[name]
    X = api.PcfSet(o, t, v, device=DEV)
    M = fn(X, window=window).cpu().numpy().astype(np.float64)
    n = len(o) - 1
    r0, r1, c0, c1 = window if window else (0, n, 0, n)
    I, J = np.meshgrid(np.arange(r0, r1), np.arange(c0, c1), indexing="ij")
    ref, ab = oracle.entries(okind, p, o, t, v, I.ravel(), J.ravel(), with_abs=True)
    ref = ref.reshape(M.shape)
    sc = _scale(okind, p, ab).reshape(M.shape)
    err = np.abs(M - ref)
    bad = err > tol * np.maximum(sc, 1e-300)
    assert not bad.any(), (name, np.argwhere(bad)[:5], err[bad][:5], ref[bad][:5])
    return M


def test_userguide_example_exact():
    g = json.load(open(os.path.join(GOLD, "userguide_4pcf.json")))
    t = np.array([r[0] for pcf in g["pcfs"] for r in pcf], dtype=np.float64)
    v = np.array([r[1] for pcf in g["pcfs"] for r in pcf], dtype=np.float64)
    o = np.concatenate([[0], np.cumsum([len(pcf) for pcf in g["pcfs"]])])
    X = api.PcfSet(o, t, v, device=DEV)
    assert np.array_equal(api.pdist(X, 1.0).cpu().numpy(), np.array(g["l1"], float))
    assert np.array_equal(api.gram(X).cpu().numpy(), np.array(g["gram"], float))
    m35 = api.pdist(X, 3.5).cpu().numpy()
    assert np.max(np.abs(m35 - np.array(g["l3_5"]))) <= 0.5e-8 + 1e-15
    for dt in (np.float32,):
        X32 = api.PcfSet(o, t.astype(dt), v.astype(dt), device=DEV)
        assert np.array_equal(api.pdist(X32, 1.0).cpu().numpy(), np.array(g["l1"], dt))
        assert np.array_equal(api.gram(X32).cpu().numpy(), np.array(g["gram"], dt))


@pytest.mark.parametrize("name", ["l1", "l2", "l2sq", "gram", "l3.5", "l3pow", "l1.5", "l2.7"])
def test_small_plain_fp64(name):
    # the small plain configuration: N = 200, counts U{10..100}
    o, t, v = workloads.config_plain_small()
    M = _check_full(name, o, t, v, 1e-12)
    assert np.array_equal(M, M.T)
    if name != "gram":
        assert np.all(np.diag(M) == 0)


@pytest.mark.parametrize("name", ["l1", "l2sq", "gram"])
def test_ragged_many_tiles(name):
    # lengths from 1 (the zero PCF) to 900: several blocks, ragged tails
    rng = np.random.default_rng(5)
    counts = rng.integers(1, 900, size=260)
    counts[::17] = 1
    P = int(counts.sum())
    o = np.concatenate([[0], np.cumsum(counts)])
    t = np.empty(P)
    v = rng.standard_normal(P)
    for i in range(len(counts)):
        a, b = o[i], o[i + 1]
        t[a:b] = np.concatenate([[0.0], np.cumsum(rng.exponential(1.0, b - a - 1))])
        v[b - 1] = 0.0
    _check_full(name, o, t, v, 1e-12)


def _dyadic_set(rng, N, nmax, grid=4, tmax=64):
    pcfs = []
    for _ in range(N):
        n = int(rng.integers(1, nmax + 1))
        ticks = np.sort(rng.choice(np.arange(1, tmax), size=min(n - 1, tmax - 1),
                                   replace=False)) / grid
        tt = np.concatenate([[0.0], ticks])
        vv = rng.integers(-8, 9, size=len(tt)) / 4.0
        vv[-1] = 0.0
        pcfs.append((tt, vv))
    o = np.concatenate([[0], np.cumsum([len(a) for a, _ in pcfs])])
    return o, np.concatenate([a for a, _ in pcfs]), np.concatenate([b for _, b in pcfs])


@pytest.mark.parametrize("name", ["l1", "l2sq", "gram", "l3pow"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_dyadic_bitwise(name, dtype):
    # many equal times across PCFs (ties) and repeated values; all arithmetic
    # exact, so any summation order gives the same bits
    rng = np.random.default_rng(7)
    o, t, v = _dyadic_set(rng, 150, 40)
    fn, okind, p = KINDS[name]
    X = api.PcfSet(o, t.astype(dtype), v.astype(dtype), device=DEV)
    M = fn(X).cpu().numpy()
    R = oracle.matrix(okind, p, o, t, v).astype(dtype)
    assert np.array_equal(M, R)


@pytest.mark.parametrize("name", ["l1", "l2", "gram", "l3.5", "l2.7"])
def test_fp32_against_rounded_inputs(name):
    o, t, v = workloads.uniform_counts(400, 50, 500, seed=21, dtype=np.float32)
    _check_full(name, o, t, v, 1e-5)


@pytest.mark.parametrize("win", [(10, 70, 40, 190), (0, 50, 100, 230), (60, 61, 0, 230),
                                 (30, 90, 30, 90), (200, 230, 0, 20), (0, 230, 0, 230)])
def test_windows(win):
    # a window is tiled on its own (block edges at its borders), so it is
    # compared with the oracle, not bit for bit with the full matrix
    o, t, v = workloads.uniform_counts(230, 1, 300, seed=9)
    _check_full("l1", o, t, v, 1e-12, window=win)
    _check_full("gram", o, t, v, 1e-12, window=win)


def test_upper_only_and_determinism():
    o, t, v = workloads.uniform_counts(230, 1, 300, seed=9)
    X = api.PcfSet(o, t, v, device=DEV)
    full = api.pdist(X, 1.0).cpu().numpy()
    # same plan, same bits: partial sums are added in a fixed order
    assert np.array_equal(api.pdist(X, 1.0).cpu().numpy(), full)
    U = api.pdist(X, 1.0, upper_only=True).cpu().numpy()
    iu = np.triu_indices(len(o) - 1)
    assert np.array_equal(U[iu], full[iu])
    il = np.tril_indices(len(o) - 1, -1)
    assert np.all(U[il] == 0)


def test_edge_cases():
    # single PCF; two one-row PCFs; identical PCFs; nonzero last value
    X = api.PcfSet(np.array([0, 1]), np.array([0.0]), np.array([0.0]), device=DEV)
    assert api.pdist(X, 1.0).cpu().numpy().tolist() == [[0.0]]
    o = np.array([0, 1, 2])
    X = api.PcfSet(o, np.array([0.0, 0.0]), np.array([0.0, 0.0]), device=DEV)
    assert np.all(api.gram(X).cpu().numpy() == 0)
    t = np.array([0.0, 1.5, 2.0, 0.0, 1.5, 2.0])
    v = np.array([1.0, -2.0, 0.0, 1.0, -2.0, 0.0])
    X = api.PcfSet(np.array([0, 3, 6]), t, v, device=DEV)
    assert np.all(api.pdist(X, 1.0).cpu().numpy() == 0)
    assert np.all(api.gram(X).cpu().numpy() == 1.5 + 4 * 0.5)
    # unbounded tail: last values differ -> +inf distance; product -> +-inf
    t = np.array([0.0, 1.0, 0.0, 1.0])
    v = np.array([1.0, 1.0, 2.0, -3.0])
    X = api.PcfSet(np.array([0, 2, 4]), t, v, device=DEV)
    D = api.pdist(X, 1.0).cpu().numpy()
    assert D[0, 1] == np.inf and D[1, 0] == np.inf and D[0, 0] == 0
    G = api.gram(X).cpu().numpy()
    assert G[0, 1] == -np.inf and G[0, 0] == np.inf and G[1, 1] == np.inf


def test_long_pcfs_global_path():
    # two very long PCFs (records do not fit one tile's LDS together) among
    # short ones: those tiles read records from global memory
    rng = np.random.default_rng(3)
    counts = np.array([30, 9000, 25, 7000, 40, 5])
    o = np.concatenate([[0], np.cumsum(counts)])
    P = int(counts.sum())
    t = np.empty(P)
    v = rng.standard_normal(P)
    for i in range(len(counts)):
        a, b = o[i], o[i + 1]
        t[a:b] = np.concatenate([[0.0], np.cumsum(rng.exponential(0.01, b - a - 1))])
        v[b - 1] = 0.0
    for name in ("l1", "l2sq", "gram"):
        _check_full(name, o, t, v, 1e-12)


def test_validation_flags_bad_pcf():
    o, t, v = workloads.uniform_counts(50, 3, 20, seed=4)
    X = api.PcfSet(o, t, v, device=DEV)
    assert api.validate(X) == -1
    t2 = t.copy()
    t2[o[7] + 1] = t2[o[7] + 2]  # equal times in PCF 7
    v2 = v.copy()
    v2[o[30] - 1] = 0.5          # nonzero last value of PCF 29
    X2 = api.PcfSet(o, t2, v2, device=DEV)
    assert api.validate(X2) == 7
    with pytest.raises(RuntimeError) as e:
        api.pdist(X2, 1.0, validate=True)
    assert "PCF_EDATA" in str(e.value) and "PCF 7" in str(e.value)
    t3 = t.copy()
    t3[o[12]] = 0.25            # first time not 0
    assert api.validate(api.PcfSet(o, t3, v, device=DEV)) == 12
    v3 = v.copy()
    v3[o[40] + 1] = np.nan
    assert api.validate(api.PcfSet(o, t, v3, device=DEV)) == 40


def test_plain_full_size_sampled():
    # the N = 20,000 configuration, FP64 L1, in the benchmark's launch
    # configuration; 3000 sampled entries plus properties of the whole matrix
    o, t, v = workloads.config_plain()
    X = api.PcfSet(o, t, v, device=DEV)
    M = api.pdist(X, 1.0)
    assert torch.equal(M, M.T)
    assert torch.all(torch.diagonal(M) == 0)
    assert torch.isfinite(M).all()
    I, J = workloads.random_pairs(X.n, 3000, seed=77)
    Mh = M[torch.as_tensor(I, device=DEV), torch.as_tensor(J, device=DEV)].cpu().numpy()
    ref = oracle.entries(oracle.LP, 1.0, o, t, v, I, J)
    assert np.all(np.abs(Mh - ref) <= 1e-12 * ref)


@pytest.mark.parametrize("n", [2, 5, 9, 13, 17, 40])
def test_tiny_tiles_few_active_lanes(n):
    # a tile with a handful of steps: most lanes idle, one lane may run both
    # of its chains with a single active lane in its wave
    rng = np.random.default_rng(n)
    for N in (2, 3):
        counts = np.full(N, n)
        o = np.concatenate([[0], np.cumsum(counts)])
        t = np.concatenate([np.concatenate([[0.0], np.cumsum(rng.exponential(1.0, n - 1))])
                            for _ in range(N)])
        v = rng.standard_normal(N * n)
        v[o[1:] - 1] = 0.0
        for name in ("l1", "l2sq", "gram"):
            _check_full(name, o, t, v, 1e-12)


def test_huge_pcf_wide_step_prefix():
    # one PCF of 2^25 rows against a block of 32 two-row PCFs: that tile's
    # step total passes 2^30 (global mode, 64-bit step prefix and lane split)
    rng = np.random.default_rng(11)
    n0 = 1 << 25
    counts = np.array([n0] + [2] * 32)
    o = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    P = int(o[-1])
    t = np.empty(P)
    v = np.empty(P)
    t[:n0] = np.concatenate([[0.0], np.cumsum(rng.exponential(1.0, n0 - 1))])
    v[:n0] = rng.standard_normal(n0)
    v[n0 - 1] = 0.0
    tmax = t[n0 - 1]
    for j in range(32):
        a = n0 + 2 * j
        t[a], t[a + 1] = 0.0, rng.uniform(0.01, 1.0) * tmax
        v[a], v[a + 1] = rng.standard_normal(), 0.0
    X = api.PcfSet(o, t, v, device=DEV)
    pick_i = np.array([0, 0, 0, 5, 9])
    pick_j = np.array([3, 17, 32, 0, 21])
    for name in ("l1", "gram"):
        fn, okind, p = KINDS[name]
        M = fn(X).cpu().numpy()
        assert np.array_equal(M, M.T), name
        ref, ab = oracle.entries(okind, p, o, t, v, pick_i, pick_j, with_abs=True)
        err = np.abs(M[pick_i, pick_j] - ref)
        assert np.all(err <= 1e-12 * np.maximum(ab, 1e-300)), (name, err, ref)


@pytest.fixture(scope="module")
def plain_sets():
    """The N = 20,000 configuration in both precisions (FP32: the FP64 draws
    rounded, duplicates dropped), resident on the GPU."""
    sets = {}
    for dt in (np.float64, np.float32):
        o, t, v = workloads.config_plain(dtype=dt)
        sets[dt] = (o, t, v, api.PcfSet(o, t, v, device=DEV))
    return sets


@pytest.mark.parametrize("name,dt,tol", [("l2", np.float64, 1e-12), ("gram", np.float64, 1e-12),
                                         ("l1", np.float32, 1e-5), ("l2", np.float32, 1e-5),
                                         ("gram", np.float32, 1e-5)])
def test_plain_full_size_sampled_kinds(plain_sets, name, dt, tol):
    # the N = 20,000 configuration at full size in the benchmark's launch
    # configuration: 3,000 random entries plus the whole first row against
    # the oracle (FP32: on the rounded inputs), and properties of the whole
    # matrix
    o, t, v, X = plain_sets[dt]
    fn, okind, p = KINDS[name]
    M = fn(X)
    assert M.dtype == X.dtype
    assert torch.equal(M, M.T)
    assert torch.isfinite(M).all()
    if okind != oracle.GRAM:
        assert torch.all(torch.diagonal(M) == 0)
    I, J = workloads.random_pairs(X.n, 3000, seed=78)
    I = np.concatenate([I, np.zeros(X.n, dtype=I.dtype)])
    J = np.concatenate([J, np.arange(X.n, dtype=J.dtype)])
    got = M[torch.as_tensor(I, device=DEV), torch.as_tensor(J, device=DEV)]
    got = got.double().cpu().numpy()
    ref, ab = oracle.entries(okind, p, o, t.astype(np.float64), v.astype(np.float64), I, J,
                             with_abs=True)
    err = np.abs(got - ref) / np.maximum(_scale(okind, p, ab), 1e-300)
    assert err.max() <= tol, (name, dt, err.max(), np.argmax(err))


def test_plan_reuse_across_dtypes_and_calls():
    # FP32 then FP64 sets sharing one offsets array and one Workspace: the
    # second call re-plans (records of another size) and matches the oracle;
    # the C layer refuses to reuse a plan made for the other dtype or for
    # another kind of call
    import ctypes
    from paper_2404_07183_amd import _lib
    o, t, v = workloads.uniform_counts(120, 2, 90, seed=31)
    X64 = api.PcfSet(o, t, v, device=DEV)
    X32 = api.PcfSet(X64.offsets_host, t.astype(np.float32), v.astype(np.float32), device=DEV)
    ws = api.Workspace(device=DEV)
    api.pdist(X32, 1.0, workspace=ws)
    M = api.pdist(X64, 1.0, workspace=ws).cpu().numpy()
    n = X64.n
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ref, ab = oracle.entries(oracle.LP, 1.0, o, t, v, I.ravel(), J.ravel(), with_abs=True)
    assert np.all(np.abs(M.ravel() - ref) <= 1e-12 * np.maximum(ab, 1e-300))
    lib = _lib.load()
    out = torch.empty((n, n), dtype=torch.float32, device=DEV)
    Xc = X32.c_struct()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.pcf_pairwise_lp(ctypes.byref(Xc), _lib.PCF_LP, 1.0, out.data_ptr(), n, None,
                             ws.ptr, ws.nbytes, _lib.PCF_REUSE_PLAN, stream)
    assert st == _lib.PCF_EINVAL and "FP64" in _lib.last_error()
    api.pairwise_backward(X64, api.PCF_LP_POW, 2.0, torch.ones((n, n), dtype=torch.float64,
                                                                device=DEV), workspace=ws)
    Xc = X64.c_struct()
    out64 = torch.empty((n, n), dtype=torch.float64, device=DEV)
    st = lib.pcf_pairwise_lp(ctypes.byref(Xc), _lib.PCF_LP, 1.0, out64.data_ptr(), n, None,
                             ws.ptr, ws.nbytes, _lib.PCF_REUSE_PLAN, stream)
    assert st == _lib.PCF_EINVAL and "pcf_pairwise_backward" in _lib.last_error()
