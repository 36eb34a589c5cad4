"""The autotuner's persistent cache and workload buckets (host logic only)."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2404_07183_amd import api, workloads


def _set(N, lo, hi, seed=0, dtype=np.float64):
    o, t, v = workloads.uniform_counts(N, lo, hi, seed, dtype)

    class S:  # the fields workload_signature reads, without a GPU
        pass
    X = S()
    X.offsets_host, X.n = o, N
    X.dtype = torch.float64 if dtype == np.float64 else torch.float32
    return X


def test_signature_buckets():
    a = api.workload_signature(_set(1100, 50, 500), api.PCF_LP, 1.0)
    b = api.workload_signature(_set(1900, 60, 480, seed=1), api.PCF_LP, 1.0)
    assert a == b  # same size, mean-row and max-row buckets
    assert api.workload_signature(_set(1100, 5, 20), api.PCF_LP, 1.0) != a  # shorter PCFs
    assert api.workload_signature(_set(5000, 50, 500), api.PCF_LP, 1.0) != a  # more PCFs
    assert api.workload_signature(_set(1100, 50, 500, dtype=np.float32), api.PCF_LP, 1.0) != a
    assert api.workload_signature(_set(1100, 50, 500), api.PCF_GRAM) != a
    assert api.workload_signature(_set(1100, 50, 500), api.PCF_LP, 2.5) != a
    so = np.array([0, 100, 300, 1000])
    s1 = api.workload_signature(_set(1000, 50, 500), api.PCF_LP, 2.0, set_offsets=so)
    assert "b1" in s1 and "n9" not in s1


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tiles.json")
    c = api.TuneCache(path)
    assert c.get("k", context="dev|x") is None  # no file yet
    times = {(32, 2): 1.5, (16, 2): 2.0, None: 1.7}
    c.put("k", (32, 2), times, context="dev|x")
    c.put("k2", None, {None: 3.0}, context="dev|x")
    assert api.TuneCache(path).get("k", context="dev|x") == ((32, 2), times)
    assert api.TuneCache(path).get("k2", context="dev|x") == (None, {None: 3.0})
    assert api.TuneCache(path).get("k", context="dev|y") is None  # another build or GPU
    assert sorted(os.listdir(os.path.dirname(path))) == ["tiles.json"]  # no temp files left
    with open(path, "w") as f:
        f.write("{not json")
    assert api.TuneCache(path).get("k", context="dev|x") is None  # unreadable: empty


def test_autotune_cache_hit_runs_nothing(tmp_path):
    # a stored entry for this library build and device is returned without
    # launching any candidate
    c = api.TuneCache(str(tmp_path / "tiles.json"))
    c.put("sig-a", (24, 2), {(24, 2): 1.0, (32, 2): 1.2})

    def run(shape):
        raise AssertionError("a cached key must not be re-tuned")
    assert api.autotune(run, "sig-a", cache=c) == ((24, 2), {(24, 2): 1.0, (32, 2): 1.2})
    with open(c.path) as f:
        assert len(json.load(f)) == 1


def test_cache_unwritable_is_not_fatal(tmp_path):
    blocker = tmp_path / "file"
    blocker.write_text("x")
    c = api.TuneCache(str(blocker / "tiles.json"))  # a directory that cannot exist
    assert c.put("k", (32, 2), {(32, 2): 1.0}, context="dev|x") is False
    assert c.get("k", context="dev|x") is None
