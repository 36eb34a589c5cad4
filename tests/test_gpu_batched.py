"""Batched problems in one persistent launch (pcf_pairwise_batched), tile
shapes, and HIP-graph replay, against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2404_07183_amd import api, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _small_batch(seed=13):
    rng = np.random.default_rng(seed)
    sizes = np.array([0, 1, 2, 37, 5, 16, 0, 64, 3, 90])
    counts = np.minimum(rng.geometric(1 / 40, size=sizes.sum()), 400)
    o = np.concatenate([[0], np.cumsum(counts)])
    t = np.empty(o[-1])
    v = rng.standard_normal(o[-1])
    for i in range(len(counts)):
        a, b = o[i], o[i + 1]
        t[a:b] = np.concatenate([[0.0], np.cumsum(rng.exponential(1.0, b - a - 1))])
        v[b - 1] = 0.0
    so = np.concatenate([[0], np.cumsum(sizes)])
    return so, o, t, v


def _sub(o, t, v, a, b):
    oo = o[a:b + 1] - o[a]
    return oo, t[o[a]:o[b]], v[o[a]:o[b]]


@pytest.mark.parametrize("kind,p,okind", [(api.PCF_LP, 1.0, oracle.LP),
                                          (api.PCF_LP, 2.0, oracle.LP),
                                          (api.PCF_GRAM, 0.0, oracle.GRAM)])
@pytest.mark.parametrize("shape", [None, (8, 2), (32, 4)])
def test_small_batch_vs_oracle(kind, p, okind, shape):
    so, o, t, v = _small_batch()
    X = api.PcfSet(o, t, v, device=DEV)
    out, oo = api.pairwise_batched(so, X, kind, p, shape=shape)
    out = out.cpu().numpy()
    for b in range(len(so) - 1):
        a, e = so[b], so[b + 1]
        s = e - a
        if s == 0:
            continue
        M = out[oo[b]:oo[b] + s * s].reshape(s, s)
        oo_, tt, vv = _sub(o, t, v, a, e)
        R, ab = [], []
        I, J = np.meshgrid(np.arange(s), np.arange(s), indexing="ij")
        R, ab = oracle.entries(okind, p, oo_, tt, vv, I.ravel(), J.ravel(), with_abs=True)
        sc = ab ** (1 / p) if (okind == oracle.LP and p != 1) else ab
        assert np.all(np.abs(M.ravel() - R) <= 1e-12 * np.maximum(sc, 1e-300)), b
        assert np.array_equal(M, M.T)


def test_batched_config_full_size_sampled():
    # the 512-problem configuration at full size (L2 distances, FP64)
    so, o, t, v = workloads.config_batched()
    X = api.PcfSet(o, t, v, device=DEV)
    out, oo = api.pairwise_batched(so, X, api.PCF_LP, 2.0)
    rng = np.random.default_rng(0)
    sizes = np.diff(so)
    for b in rng.choice(len(sizes), size=24, replace=False):
        s = int(sizes[b])
        M = out[int(oo[b]):int(oo[b]) + s * s].view(s, s)
        assert torch.equal(M, M.T)
        assert torch.all(torch.diagonal(M) == 0)
        I = rng.integers(0, s, size=40)
        J = rng.integers(0, s, size=40)
        got = M[torch.as_tensor(I, device=DEV), torch.as_tensor(J, device=DEV)].cpu().numpy()
        oo_, tt, vv = _sub(o, t, v, so[b], so[b + 1])
        ref, ab = oracle.entries(oracle.LP, 2.0, oo_, tt, vv, I, J, with_abs=True)
        assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(np.sqrt(ab), 1e-300)), b


def test_batched_graph_replay():
    # a call that reuses its plan only launches kernels: capture it in a HIP
    # graph and replay; every replay must equal the eager result bit for bit
    so, o, t, v = _small_batch(21)
    X = api.PcfSet(o, t, v, device=DEV)
    ws = api.Workspace(device=DEV)
    out = torch.zeros(int((np.diff(so) ** 2).sum()), dtype=torch.float64, device=DEV)
    api.pairwise_batched(so, X, api.PCF_LP, 1.0, out=out, workspace=ws)
    eager = out.clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            api.pairwise_batched(so, X, api.PCF_LP, 1.0, out=out, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager)
        _ = (X.t * 2).sum().item()  # unrelated eager work between replays


def test_batch_with_range_and_weight_vs_oracle():
    # bounds and a time weight: each problem's matrix against the oracle's
    # weighted integrals over the range
    so, o, t, v = _small_batch()
    X = api.PcfSet(o, t, v, device=DEV)
    a, b, c = 1.5, 30.0, 0.2
    out, oo = api.pairwise_batched(so, X, api.PCF_LP, 1.0, bounds=(a, b), weight=("exp", c))
    out = out.cpu().numpy()
    for k in range(len(so) - 1):
        s = so[k + 1] - so[k]
        if s == 0:
            continue
        M = out[oo[k]:oo[k] + s * s].reshape(s, s)
        oo_, tt, vv = _sub(o, t, v, so[k], so[k + 1])
        I, J = np.meshgrid(np.arange(s), np.arange(s), indexing="ij")
        R, ab = oracle.entries_w(oracle.LP, 1.0, oracle.W_EXP, c, oo_, tt, vv, I.ravel(),
                                 J.ravel(), a=a, b=b, with_abs=True)
        assert np.all(np.abs(M.ravel() - R) <= 1e-12 * np.maximum(ab, 1e-300)), k


def test_autotune_persists_across_processes(tmp_path):
    # the first tuning runs every candidate and stores the winner for this
    # library build and GPU; a later process (the in-process memo cleared)
    # takes it from the file without launching anything
    so, o, t, v = workloads.config_batched(B=16, smax=64, mean_len=40)
    X = api.PcfSet(o, t, v, device=DEV)
    sizes = np.diff(so)
    out = torch.empty(int((sizes ** 2).sum()), dtype=torch.float64, device=DEV)
    ws = api.Workspace(device=DEV)
    calls = []

    def run(shape):
        calls.append(shape)
        api.pairwise_batched(so, X, api.PCF_LP, 2.0, out=out, workspace=ws, shape=shape)
    key = api.workload_signature(X, api.PCF_LP, 2.0, set_offsets=so)
    cache = api.TuneCache(str(tmp_path / "tiles.json"))
    shape, times = api.autotune(run, key, cache=cache, reps=2)
    assert len(calls) == 3 * len(api.TILE_SHAPES) and shape in api.TILE_SHAPES
    assert set(times) == set(api.TILE_SHAPES)
    api._TUNED.clear()
    calls.clear()
    assert api.autotune(run, key, cache=api.TuneCache(cache.path)) == (shape, times)
    assert calls == []
