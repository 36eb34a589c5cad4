"""CPU-side checks of the HIP library: it loads, exports every symbol that
include/pcf.h declares, rejects bad arguments before touching a device, and
its host planner tiles the matrix as documented. No GPU compute runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2404_07183_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "pcf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pcf_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _header_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.exported_names(), name
    assert lib.pcf_abi_version() == 1


def test_argument_errors_need_no_device():
    lib = _lib.load()
    # NULL set
    st = lib.pcf_pairwise_lp(None, _lib.PCF_LP, 1.0, None, 1, None, None, 0, 0, None)
    assert st == _lib.PCF_EINVAL
    assert "NULL" in _lib.last_error()
    X = _lib.pcf_set(0, None, None, None, _lib.PCF_F64, None)
    # p < 1 and non-finite p
    for p in (0.5, float("nan"), float("inf")):
        st = lib.pcf_pairwise_lp(ctypes.byref(X), _lib.PCF_LP, p, None, 1, None, None, 0, 0, None)
        assert st == _lib.PCF_EINVAL
    # wrong kind for pcf_pairwise_lp
    st = lib.pcf_pairwise_lp(ctypes.byref(X), _lib.PCF_GRAM, 1.0, None, 1, None, None, 0, 0, None)
    assert st == _lib.PCF_EINVAL
    # empty set is a no-op
    st = lib.pcf_pairwise_lp(ctypes.byref(X), _lib.PCF_LP, 1.0, None, 1, None, None, 0, 0, None)
    assert st == _lib.PCF_OK
    st = lib.pcf_gram(ctypes.byref(X), None, 1, None, None, 0, 0, None)
    assert st == _lib.PCF_OK
    # bad dtype
    Xb = _lib.pcf_set(0, None, None, None, 7, None)
    assert lib.pcf_gram(ctypes.byref(Xb), None, 1, None, None, 0, 0, None) == _lib.PCF_EINVAL
    # n < 0
    Xn = _lib.pcf_set(-1, None, None, None, _lib.PCF_F64, None)
    assert lib.pcf_gram(ctypes.byref(Xn), None, 1, None, None, 0, 0, None) == _lib.PCF_EINVAL
    # integration ranges and time weights are checked before any device work
    for a, b in ((2.0, 2.0), (-1.0, 3.0), (3.0, 1.0), (float("nan"), 1.0)):
        assert lib.pcf_restrict_rows(ctypes.byref(X), a, b, None, None, None) == _lib.PCF_EINVAL
    bad_weights = ((0, 1.0), (_lib.PCF_WEIGHT_EXP, 0.0), (_lib.PCF_WEIGHT_EXP, float("inf")),
                   (_lib.PCF_WEIGHT_POW, -1.0), (_lib.PCF_WEIGHT_POW, float("nan")))
    for wk, c in bad_weights:
        assert lib.pcf_warp_rows(ctypes.byref(X), wk, c, None, None, None) == _lib.PCF_EINVAL
        assert lib.pcf_warp(ctypes.byref(X), wk, c, None, None, None, None) == _lib.PCF_EINVAL
    assert lib.pcf_warp(ctypes.byref(X), _lib.PCF_WEIGHT_EXP, 1.0, None, None, None,
                        None) == _lib.PCF_OK
    # the gradient maps through a restriction and a warp check the same
    # arguments as the forward calls, and NULL pointers, before device work
    for a, b in ((2.0, 2.0), (-1.0, 3.0), (3.0, 1.0)):
        assert lib.pcf_restrict_backward(ctypes.byref(X), a, b, None, None, None, None, None,
                                         None) == _lib.PCF_EINVAL
    for wk, c in bad_weights:
        assert lib.pcf_warp_backward(ctypes.byref(X), wk, c, None, None, None, None, None,
                                     None) == _lib.PCF_EINVAL
    X1 = _lib.pcf_set(1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8),
                      _lib.PCF_F64, None)  # (never dereferenced: refused first)
    assert lib.pcf_restrict_backward(ctypes.byref(X1), 0.5, 2.0, None, None, None, None,
                                     None, None) == _lib.PCF_EINVAL
    assert lib.pcf_warp_backward(ctypes.byref(X1), _lib.PCF_WEIGHT_EXP, 1.0, None, None,
                                 None, None, None, None) == _lib.PCF_EINVAL
    assert lib.pcf_restrict_backward(ctypes.byref(X), 0.5, 2.0, None, None, None, None,
                                     None, None) == _lib.PCF_OK  # empty set: no-op


def _inspect(offsets, dtype=_lib.PCF_F64, window=None, backward=False):
    o = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(o) - 1
    buf = np.zeros(n + 2, dtype=np.int32)
    nb, ns, nt = _lib.pcf_plan_inspect(n, o.ctypes.data, dtype,
                                       _lib.pcf_window(*window) if window else None,
                                       backward, len(buf), buf.ctypes.data)
    return nb, ns, nt, buf[:nb + 1]


def test_planner_full_matrix_blocks():
    rng = np.random.default_rng(0)
    counts = rng.integers(1, 600, size=500)
    o = np.concatenate([[0], np.cumsum(counts)])
    for dtype, rec, bwd in [(_lib.PCF_F64, 16, False), (_lib.PCF_F32, 8, False),
                            (_lib.PCF_F64, 16, True), (_lib.PCF_F32, 8, True)]:
        nb, ns, nt, blocks = _inspect(o, dtype, backward=bwd)
        # LDS record area of a tile: half the records that fit (the adjoint's
        # 144 KiB hold records with 16 bytes of gradient slots each, in
        # multiples of 64 records)
        budget = ((144 * 1024 // (rec + 16)) // 64 * 64 if bwd else 136 * 1024 // rec) // 2
        assert blocks[0] == 0 and blocks[-1] == 500
        assert np.all(np.diff(blocks) >= 1) and np.all(np.diff(blocks) <= 32)
        for a, b in zip(blocks[:-1], blocks[1:]):
            recs = int(np.sum(counts[a:b] + 7))
            assert recs <= budget or b - a == 1
            # greedy: the next PCF would not have fitted
            if b < 500 and b - a < 32:
                assert recs + counts[b] + 7 > budget
        assert ns == 1 and nt == nb * (nb + 1) // 2


def test_planner_windows_cover_each_pair_once():
    rng = np.random.default_rng(1)
    counts = rng.integers(1, 300, size=200)
    o = np.concatenate([[0], np.cumsum(counts)])
    for win in [(0, 200, 0, 200), (10, 70, 40, 190), (0, 50, 100, 200), (60, 61, 0, 200),
                (30, 90, 30, 90)]:
        nb, ns, nt, blocks = _inspect(o, window=win)
        r0, r1, c0, c1 = win
        for cut in (r0, r1, c0, c1):
            assert cut in set(blocks.tolist())
        assert nt >= 1 and ns >= 1


def test_planner_rejects_empty_pcf():
    o = np.array([0, 3, 3, 5], dtype=np.int64)
    with pytest.raises(_lib.PcfError) as e:
        _inspect(o)
    assert "no rows" in str(e.value)


def test_planner_rejects_pcf_with_2_pow_30_rows():
    # only the offsets are read: a PCF of 2^30 rows is refused (a pair's
    # merge steps must stay below 2^31), one row fewer is accepted
    o = np.array([0, 3, 3 + (1 << 30)], dtype=np.int64)
    with pytest.raises(_lib.PcfError) as e:
        _inspect(o)
    assert "2^30" in str(e.value)
    nb, ns, nt, blocks = _inspect(np.array([0, 3, 2 + (1 << 30)], dtype=np.int64))
    assert nt >= 1


def test_reduction_and_combination_arguments_need_no_device():
    lib = _lib.load()
    X = _lib.pcf_set(0, None, None, None, _lib.PCF_F64, None)
    size = ctypes.c_size_t(0)
    g = np.array([0], dtype=np.int64)
    # unknown ops
    assert lib.pcf_reduce_workspace_bytes(ctypes.byref(X), 0, g.ctypes.data, 9,
                                          ctypes.byref(size)) == _lib.PCF_EINVAL
    assert lib.pcf_combine_workspace_bytes(ctypes.byref(X), ctypes.byref(X), 9,
                                           ctypes.byref(size)) == _lib.PCF_EINVAL
    # the empty set reduces to no groups and combines to nothing
    assert lib.pcf_reduce_workspace_bytes(ctypes.byref(X), 0, g.ctypes.data,
                                          _lib.PCF_REDUCE_MEAN, ctypes.byref(size)) == _lib.PCF_OK
    assert lib.pcf_combine_workspace_bytes(ctypes.byref(X), ctypes.byref(X),
                                           _lib.PCF_COMBINE_SUM, ctypes.byref(size)) == _lib.PCF_OK
    # groups that do not cover the set, negative B, NULL groups
    g2 = np.array([0, 1], dtype=np.int64)
    assert lib.pcf_reduce_workspace_bytes(ctypes.byref(X), 1, g2.ctypes.data,
                                          _lib.PCF_REDUCE_SUM, ctypes.byref(size)) == _lib.PCF_EINVAL
    assert lib.pcf_reduce_workspace_bytes(ctypes.byref(X), -1, g.ctypes.data,
                                          _lib.PCF_REDUCE_SUM, ctypes.byref(size)) == _lib.PCF_EINVAL
    assert lib.pcf_reduce_workspace_bytes(ctypes.byref(X), 1, None, _lib.PCF_REDUCE_SUM,
                                          ctypes.byref(size)) == _lib.PCF_EINVAL
    # different dtypes
    Xf = _lib.pcf_set(0, None, None, None, _lib.PCF_F32, None)
    assert lib.pcf_combine_workspace_bytes(ctypes.byref(X), ctypes.byref(Xf),
                                           _lib.PCF_COMBINE_SUM, ctypes.byref(size)) == _lib.PCF_EINVAL


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_out_tensors_are_checked_before_the_library_is_called(monkeypatch):
    """A short, wrongly placed or wrongly typed out tensor is refused on the
    host, before any library call (the C ABI only sees ldo)."""
    import torch
    from paper_2404_07183_amd import _lib, api

    def no_call(*a, **k):  # any library call would be a failure here
        raise AssertionError("library called")

    monkeypatch.setattr(_lib, "pcf_pairwise_lp", no_call, raising=False)
    monkeypatch.setattr(_lib, "pcf_gram", no_call, raising=False)
    monkeypatch.setattr(_lib, "pcf_cross", no_call, raising=False)
    monkeypatch.setattr(_lib, "pcf_pairwise_batched", no_call, raising=False)
    monkeypatch.setattr(_lib, "pcf_workspace_bytes", lambda *a: 256, raising=False)
    monkeypatch.setattr(_lib, "pcf_cross_workspace_bytes", lambda *a: 256, raising=False)
    monkeypatch.setattr(_lib, "pcf_batched_workspace_bytes", lambda *a: 256, raising=False)
    o = np.array([0, 2, 5, 7], dtype=np.int64)
    t = np.array([0, 1, 0, 1, 2, 0, 3], dtype=np.float64)
    v = np.array([1, 0, 2, 1, 0, 5, 0], dtype=np.float64)
    X = api.PcfSet(o, t, v, device="cpu")
    ws = api.Workspace(device="cpu")
    with pytest.raises(ValueError, match="shape"):
        api.pdist(X, out=torch.zeros((2, 3), dtype=torch.float64), workspace=ws)
    with pytest.raises(ValueError, match="shape"):
        api.gram(X, window=(0, 3, 1, 3), out=torch.zeros((3, 1), dtype=torch.float64),
                 workspace=ws)
    with pytest.raises(ValueError, match="device"):
        api.pdist(X, out=torch.zeros((3, 3), dtype=torch.float64, device="meta"),
                  workspace=ws)
    with pytest.raises(ValueError, match="dtype"):
        api.pdist(X, out=torch.zeros((3, 3), dtype=torch.float32), workspace=ws)
    with pytest.raises(ValueError, match="shape"):
        api.cdist(X, X, out=torch.zeros((3, 2), dtype=torch.float64), workspace=ws)
    with pytest.raises(ValueError, match="need"):
        api.pairwise_batched([0, 1, 3], X, out=torch.zeros(4, dtype=torch.float64),
                             workspace=ws)


def test_plan_key_separates_dtypes(monkeypatch):
    """Two sets sharing one offsets array but differing in dtype never reuse
    each other's plan through one Workspace (the record size differs): the
    second call must not pass PCF_REUSE_PLAN; a repeat call on the same set
    does."""
    import torch
    from paper_2404_07183_amd import _lib, api
    seen = []

    def fake_lp(Xc, kind, p, out, ldo, win, ws, nbytes, flags, stream):
        seen.append((Xc.dtype, bool(flags & _lib.PCF_REUSE_PLAN)))
        return 0

    monkeypatch.setattr(_lib, "pcf_pairwise_lp", fake_lp, raising=False)
    monkeypatch.setattr(_lib, "pcf_workspace_bytes", lambda *a: 256, raising=False)
    monkeypatch.setattr(api, "_stream_handle", lambda s=None: None)
    o = np.array([0, 2, 5], dtype=np.int64)
    t = np.array([0, 1, 0, 1, 2], dtype=np.float64)
    v = np.array([1, 0, 2, 1, 0], dtype=np.float64)
    X64 = api.PcfSet(o, t, v, device="cpu")
    X32 = api.PcfSet(X64.offsets_host, t.astype(np.float32), v.astype(np.float32),
                     device="cpu")
    assert X32.offsets_host is X64.offsets_host
    ws = api.Workspace(device="cpu")
    api.pdist(X32, workspace=ws)
    api.pdist(X64, workspace=ws)
    api.pdist(X64, workspace=ws)
    assert seen == [(_lib.PCF_F32, False), (_lib.PCF_F64, False), (_lib.PCF_F64, True)]


def test_noalloc_refuses_oversized_sets_before_device_work():
    """pcf_pairwise_lp_noalloc sizes the call's plan on the host (offsets_host
    given) and refuses one beyond the library's array with PCF_ENOMEM before
    touching a device; it refuses plan reuse; it exports the array's size."""
    lib = _lib.load()
    n = 40000
    counts = np.full(n, 200, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced on these paths
    X = _lib.pcf_set(n, fake, fake, fake, _lib.PCF_F64, off.ctypes.data)
    st = lib.pcf_pairwise_lp_noalloc(ctypes.byref(X), _lib.PCF_LP, 1.0, fake, n, None, 0, None)
    assert st == _lib.PCF_ENOMEM
    assert "scratch" in _lib.last_error() and str(64 << 20) in _lib.last_error()
    st = lib.pcf_pairwise_lp_noalloc(ctypes.byref(X), _lib.PCF_LP, 1.0, fake, n, None,
                                     _lib.PCF_REUSE_PLAN, None)
    assert st == _lib.PCF_EINVAL
    src = open(os.path.join(ROOT, "include", "pcf.h")).read()
    assert "#define PCF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)" in src


def test_backward_deterministic_size_limit():
    """PCF_DETERMINISTIC on the adjoint bounds its pair weights over a grid of
    32 x 32 blocks (at most 65,535 a side): larger sets are refused before
    any device work."""
    lib = _lib.load()
    n = 65535 * 32 + 1
    off = np.arange(n + 1, dtype=np.int64) * 2
    fake = ctypes.c_void_p(0x1000)
    X = _lib.pcf_set(n, fake, fake, fake, _lib.PCF_F64, off.ctypes.data)
    st = lib.pcf_pairwise_backward(ctypes.byref(X), _lib.PCF_LP, 1.0, fake, n, None, 0, fake,
                                   fake, fake, 1 << 20, _lib.PCF_DETERMINISTIC, None)
    assert st == _lib.PCF_EUNSUPPORTED
    assert "DETERMINISTIC" in _lib.last_error()


def test_plan_reuse_refused_without_a_matching_plan():
    """PCF_REUSE_PLAN on a workspace this library never planned into is
    refused before any device work."""
    lib = _lib.load()
    off = np.array([0, 2, 4], dtype=np.int64)
    fake = ctypes.c_void_p(0x2000)
    ws = ctypes.c_void_p(0x7000)  # never planned into
    X = _lib.pcf_set(2, fake, fake, fake, _lib.PCF_F64, off.ctypes.data)
    st = lib.pcf_pairwise_lp(ctypes.byref(X), _lib.PCF_LP, 1.0, fake, 2, None, ws, 1 << 20,
                             _lib.PCF_REUSE_PLAN, None)
    assert st == _lib.PCF_EINVAL and "holds no plan" in _lib.last_error()
