"""The strip configuration: the 500,000 stable-rank-like PCFs (FP32, many
repeated values and non-minimal discretizations), windows of the L1 matrix
as bench.py computes them (the diagonal block as a symmetric window, the rest
as rectangles), sampled entries against the oracle on the FP32 inputs."""
import numpy as np
import pytest
import torch

import oracle
from paper_2404_07183_amd import api, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def strip_set():
    o, t, v = workloads.config_strip()
    return o, t, v, api.PcfSet(o, t, v, device=DEV)


@pytest.mark.parametrize("win", [(0, 3000, 0, 3000), (0, 2000, 100000, 102500),
                                 (60000, 62500, 499000, 500000)])
def test_strip_windows_sampled(strip_set, win):
    o, t, v, X = strip_set
    r0, r1, c0, c1 = win
    W = api.pdist(X, 1.0, window=win)
    assert W.shape == (r1 - r0, c1 - c0) and torch.isfinite(W).all()
    # 34,000 random entries per window (over 10^5 in all) and the window's
    # whole first row
    rng = np.random.default_rng(r0 + c0)
    I = np.concatenate([rng.integers(r0, r1, size=34000), np.full(c1 - c0, r0)])
    J = np.concatenate([rng.integers(c0, c1, size=34000), np.arange(c0, c1)])
    got = W[torch.as_tensor(I - r0, device=DEV), torch.as_tensor(J - c0, device=DEV)]
    got = got.cpu().numpy().astype(np.float64)
    ref = oracle.entries(oracle.LP, 1.0, o, t, v, I, J)
    err = np.abs(got - ref) / np.maximum(ref, 1e-30)
    assert err.max() <= 1e-5, (win, err.max())
    if r0 == c0 and r1 == c1:
        assert torch.equal(W, W.T)
        assert torch.all(torch.diagonal(W) == 0)


def test_strip_first_row_whole(strip_set):
    # row 0 of the strip over all 500,000 columns (a one-row window), every
    # entry against the oracle
    o, t, v, X = strip_set
    W = api.pdist(X, 1.0, window=(0, 1, 0, X.n))
    assert W.shape == (1, X.n)
    got = W[0].cpu().numpy().astype(np.float64)
    J = np.arange(X.n)
    ref = oracle.entries(oracle.LP, 1.0, o, t, v, np.zeros_like(J), J)
    err = np.abs(got - ref) / np.maximum(ref, 1e-30)
    assert got[0] == 0.0 and err.max() <= 1e-5, err.max()
