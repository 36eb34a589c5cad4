"""Benchmark of the PCF pairwise-matrix hot path on one MI355X.

Default workload: the L1 distance matrix, FP64, of N = 20,000 synthetic PCFs
(row counts uniform on 50..500, Exp(1) gaps, N(0,1) values, last value 0).
One step = one full call (tile plan reused from the workspace, breakpoint
records packed, every pair integral computed and both triangles written)
with inputs resident in HBM. Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

The JSON carries the whole-call throughput (pair integrals per second over
the N(N-1)/2 upper-triangle pairs), the dominant kernel's roofline entry
(FP64 VALU lane-operations; its duration from HIP events around calls that
only launch the tile kernel) and the CPU oracle timed on a bounded sample on
this host's cores. Unless --no-extras, it also carries the extra lines:
batched (512 independent matrices), fwd_bwd (forward + adjoint), cross
(10,000 x 20,000 cross-set matrix), single (L2 norms) and reduce (mean and
std by reduction trees), bounded_weighted (L1 over a range with a time
weight), small (per-call latency of the 200-PCF matrix). Every line carries
its parity against the oracle as max, 99th percentile and median of the
error over the entry's scale. --only NAME[,NAME] runs extra lines alone (also
general_p: d_p^p for p = 3, 3.5, 2.7 in both precisions);
--config strip the 62,500 x 500,000 strip of the 500,000-PCF set.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_LANE_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock
OPS_PER_STEP = {"l1": 4, "l2sq": 5, "l2": 5, "gram": 4}  # algorithmic FP64 ops
# algorithmic FP64 ops of one adjoint step: compare, width, the two value
# derivatives accumulated (d_2^2: a difference, two scaled FMAs; Gram: two
# FMAs), the time derivative of the ending breakpoint (d_2^2: two squared
# differences, their difference; Gram: a difference and a product) weighted
# and accumulated
ADJ_OPS = {"l2sq": 12, "gram": 8}


# the sources the tile kernel, its launch arguments and its plan are built from
TILE_SOURCES = ("common.hpp", "kernels.hip", "launch.hpp", "plan.cpp", "plan.hpp", "tile.hpp")


def kernel_source_digest():
    """SHA-256 over the tile kernel's sources (file names and contents, in
    TILE_SOURCES order): identifies the kernel build that counters were
    taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2404_07183_amd", "csrc")
    for name in TILE_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(key):
    """HBM bytes per launch of the tile kernel for workload `key`, from the
    committed counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by the
    same counter's reading for a copy of known size); None when there is no
    entry or the sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    entry = data.get("entries", {}).get(key)
    if not entry or entry.get("source_sha256") != kernel_source_digest():
        return None
    return entry.get("bytes_per_launch")


def err_stats(err):
    """max, 99th percentile and median of per-entry errors over their scale."""
    err = np.asarray(err, dtype=np.float64)
    return {"max_error_over_scale": float(err.max()),
            "p99_error_over_scale": float(np.percentile(err, 99)),
            "median_error_over_scale": float(np.median(err))}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def merge_steps_full(o):
    """sum over pairs i<j of (n_i - 1) + (n_j - 1): finite cells without ties."""
    n = np.diff(o).astype(np.float64)
    N = len(n)
    return float((N - 1) * np.sum(n - 1))


def cpu_baseline(o, t, v, kind_name, seconds=12.0, seed=123):
    """The oracle, as it stands, on random pairs of the same workload, run on
    all host cores (one thread per core; each ctypes call releases the GIL).
    Returns pairs/s, the number of pairs timed, the thread count, the wall
    time, and the pairs with their oracle values and sums of |h|·width."""
    import concurrent.futures as cf

    import oracle
    from paper_2404_07183_amd import workloads

    kind, p = {"l1": (oracle.LP, 1.0), "l2": (oracle.LP, 2.0), "l2sq": (oracle.LP_POW, 2.0),
               "gram": (oracle.GRAM, 0.0)}[kind_name]
    # host threads: the cores this process may run on, at most 16 (the host
    # share that comes with one GPU on the machines this runs on)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 16))
    N = len(o) - 1
    # one thread: the single-thread rate, also used to size the sample
    I, J = workloads.random_pairs(N, 4000, seed=seed)
    t0 = time.perf_counter()
    oracle.entries(kind, p, o, t, v, I, J)
    per_pair = (time.perf_counter() - t0) / len(I)
    chunk = max(1, int(seconds / per_pair))
    I, J = workloads.random_pairs(N, chunk * cores, seed=seed + 1)
    parts = [(I[k * chunk:(k + 1) * chunk], J[k * chunk:(k + 1) * chunk]) for k in range(cores)]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        got = list(ex.map(lambda ij: oracle.entries(kind, p, o, t, v, ij[0], ij[1],
                                                    with_abs=True), parts))
    dt = time.perf_counter() - t0
    ref = np.concatenate([g[0] for g in got])
    ab = np.concatenate([g[1] for g in got])
    return len(I) / dt, len(I), cores, dt, (I, J, ref, ab), 1.0 / per_pair


def run_plain(args):
    import torch

    from paper_2404_07183_amd import api, workloads

    dtype = np.float64 if args.dtype == "f64" else np.float32
    o, t, v = workloads.config_plain(dtype=dtype, N=args.n)
    X = api.PcfSet(o, t, v, device="cuda:0")
    N = X.n
    fn = {"l1": lambda **k: api.pdist(X, 1.0, **k),
          "l2": lambda **k: api.pdist(X, 2.0, **k),
          "l2sq": lambda **k: api.pdist(X, 2.0, power=True, **k),
          "gram": lambda **k: api.gram(X, **k)}[args.kind]
    out = torch.empty((N, N), dtype=X.dtype, device="cuda:0")
    ws = api.Workspace(device="cuda:0")
    for _ in range(args.warmup):
        fn(out=out, workspace=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        fn(out=out, workspace=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_step = e0.elapsed_time(e1) / args.steps
    # dominant kernel alone: same calls with the records already packed, so
    # each call launches only the counter reset and the tile kernel
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    k0.record(stream)
    for _ in range(args.steps):
        fn(out=out, workspace=ws, packed=True)
    k1.record(stream)
    torch.cuda.synchronize()
    ms_kernel = k0.elapsed_time(k1) / args.steps
    pairs = N * (N - 1) / 2
    steps = merge_steps_full(o)
    ops = steps * OPS_PER_STEP[args.kind]
    achieved = ops / (ms_kernel * 1e-3)
    res = {
        "metric": "PCF pair-integrals/sec (%s, %s)" % (args.kind.upper(), args.dtype.upper()),
        "value": pairs / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": "plain %s distance matrix: N=%d PCFs, counts U{50..500}, Exp(1) gaps, "
                        "N(0,1) values, last value 0, %s; full symmetric output" % (
                            args.kind.upper(), N, args.dtype.upper()),
            "n_pcf": N, "rows": int(o[-1]), "pairs": pairs, "merge_steps": steps,
        },
        "merge_steps_per_s": steps / (ms_step * 1e-3),
        "wall_s": wall,
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP64_LANE_OPS / 1e12,
            "unit": "TOP/s",
            "frac": achieved / PEAK_FP64_LANE_OPS,
            "traffic": measured_traffic("plain-%s-%s-n%d" % (args.kind, args.dtype, N)),
            "kernel": "pairwise_tiles<%s,%s>" % ("double" if args.dtype == "f64" else "float",
                                                  args.kind),
            "kernel_ms": ms_kernel,
            "ops_per_step": OPS_PER_STEP[args.kind],
        },
    }
    if not args.no_cpu:
        pps, npairs, cores, dt, (I, J, ref, ab), pps1 = cpu_baseline(o, t, v, args.kind)
        res["cpu_baseline"] = {"value": pps, "unit": "pairs/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "%d random pairs of the same workload, %.1f s on %d "
                                         "host threads" % (npairs, dt, cores),
                               "single_thread_value": pps1,
                               "single_thread_merge_steps_per_s": pps1 * steps / pairs,
                               "cpu_model": cpu_model()}
        # the same pairs of the benchmarked matrix against the oracle: error
        # over the scale sum |h|·width (its p-th root for d_p)
        got = out[torch.as_tensor(I, device="cuda:0"),
                  torch.as_tensor(J, device="cuda:0")].double().cpu().numpy()
        root = {"l1": 1.0, "l2": 2.0, "l2sq": 1.0, "gram": 1.0}[args.kind]
        scale = np.maximum(ab, 1e-300) ** (1.0 / root)
        err = np.abs(got - ref) / scale
        res["parity"] = dict(pairs=int(len(I)), **err_stats(err),
                             tolerance=1e-12 if args.dtype == "f64" else 1e-5,
                             reference="oracle on the cpu_baseline pairs")
    return res


def _events_ms(fn, steps, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def run_batched(steps, warmup, plain_steps_per_s=None):
    """512 independent L2 distance matrices (FP64) in one persistent launch,
    tile shape picked by the autotuner, replayed as a HIP graph."""
    import torch

    from paper_2404_07183_amd import api, workloads

    so, o, t, v = workloads.config_batched()
    X = api.PcfSet(o, t, v, device="cuda:0")
    sizes = np.diff(so)
    out = torch.empty(int((sizes ** 2).sum()), dtype=torch.float64, device="cuda:0")
    ws = api.Workspace(device="cuda:0")
    stream = torch.cuda.current_stream()
    # tuned per workload bucket; the choice persists across runs on this
    # machine (for this library build and GPU)
    shape, times = api.autotune(
        lambda sh: api.pairwise_batched(so, X, api.PCF_LP, 2.0, out=out, workspace=ws, shape=sh),
        key=api.workload_signature(X, api.PCF_LP, 2.0, set_offsets=so), cache=True)
    call = lambda: api.pairwise_batched(so, X, api.PCF_LP, 2.0, out=out, workspace=ws,
                                        shape=shape)
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    ms_eager = _events_ms(call, steps, stream)
    # the same call captured once and replayed
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(stream)
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            call()
    stream.wait_stream(s)
    torch.cuda.synchronize()
    ms_graph = _events_ms(g.replay, steps, stream)
    # the tile kernel alone (plan reused, records already packed)
    ms_kernel = _events_ms(lambda: api.pairwise_batched(so, X, api.PCF_LP, 2.0, out=out,
                                                        workspace=ws, shape=shape, packed=True),
                           steps, stream)
    pairs = float(np.sum(sizes * (sizes - 1) / 2))
    n = np.diff(o).astype(np.float64)
    msteps = 0.0
    for b in range(len(sizes)):
        nb = n[so[b]:so[b + 1]]
        msteps += (len(nb) - 1) * np.sum(nb - 1)
    ms = min(ms_eager, ms_graph)
    # sampled parity: 3,000 random entries over the problems, by pair count
    import oracle
    rng = np.random.default_rng(31)
    npb = sizes * (sizes - 1) // 2
    bsel = rng.choice(len(sizes), size=3000, p=npb / npb.sum())
    li = np.array([rng.integers(0, sizes[b]) for b in bsel])
    lj = np.array([rng.integers(0, sizes[b]) for b in bsel])
    oo = np.zeros(len(sizes), dtype=np.int64)
    oo[1:] = np.cumsum(sizes[:-1] ** 2)
    flat = oo[bsel] + li * sizes[bsel] + lj
    got = out[torch.as_tensor(flat, device="cuda:0")].cpu().numpy()
    ref, ab = oracle.entries(oracle.LP, 2.0, o, t, v, so[bsel] + li, so[bsel] + lj,
                             with_abs=True)
    err = np.abs(got - ref) / np.maximum(np.sqrt(ab), 1e-300)
    ops = msteps * OPS_PER_STEP["l2"]
    res = {"workload": "512 independent L2 distance matrices, sizes round(exp(U(ln16,ln2048))), "
                       "counts Geometric(1/200) capped 5000, FP64",
           "problems": int(len(sizes)), "pcfs": int(X.n), "pairs": pairs, "merge_steps": msteps,
           "ms_per_step_eager": ms_eager, "ms_per_step_graph": ms_graph,
           "pairs_per_s": pairs / (ms * 1e-3), "merge_steps_per_s": msteps / (ms * 1e-3),
           "tile_shape": list(shape) if shape else None,
           "autotune_ms": {str(k): v for k, v in times.items()},
           "roofline": {"bound": "alu", "achieved": ops / (ms_kernel * 1e-3) / 1e12,
                        "peak": PEAK_FP64_LANE_OPS / 1e12, "unit": "TOP/s",
                        "frac": ops / (ms_kernel * 1e-3) / PEAK_FP64_LANE_OPS,
                        "kernel": "pairwise_tiles<double,l2>", "kernel_ms": ms_kernel,
                        "ops_per_step": OPS_PER_STEP["l2"]},
           "parity": dict(pairs=3000, **err_stats(err), tolerance=1e-12)}
    if plain_steps_per_s:
        res["vs_plain_merge_steps_per_s"] = res["merge_steps_per_s"] / plain_steps_per_s
    return res


def run_cross(steps, warmup, plain_steps_per_s=None):
    """Cross-set L1 matrix (FP64): 10,000 query PCFs x 20,000 reference PCFs
    of the plain recipe (counts U{50..500}), each call planning, packing both
    sets and computing the rectangle; parity of a sample against the oracle."""
    import torch

    import oracle
    from paper_2404_07183_amd import api, workloads

    xs = workloads.uniform_counts(10000, 50, 500, seed=41)
    ys = workloads.uniform_counts(20000, 50, 500, seed=42)
    X = api.PcfSet(*xs, device="cuda:0")
    Y = api.PcfSet(*ys, device="cuda:0")
    out = torch.empty((X.n, Y.n), dtype=torch.float64, device="cuda:0")
    ws = api.Workspace(device="cuda:0")
    stream = torch.cuda.current_stream()
    call = lambda: api.cdist(X, Y, 1.0, out=out, workspace=ws)
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    ms = _events_ms(call, steps, stream)
    nx_ = np.diff(xs[0]).astype(np.float64)
    ny_ = np.diff(ys[0]).astype(np.float64)
    msteps = len(ny_) * np.sum(nx_ - 1) + len(nx_) * np.sum(ny_ - 1)
    pairs = float(X.n) * Y.n
    # sampled parity against the oracle on one CSR of X then Y
    rng = np.random.default_rng(43)
    I = rng.integers(0, X.n, 2000)
    J = rng.integers(0, Y.n, 2000)
    o = np.concatenate([xs[0], xs[0][-1] + ys[0][1:]])
    ref, ab = oracle.entries(oracle.LP, 1.0, o, np.concatenate([xs[1], ys[1]]),
                             np.concatenate([xs[2], ys[2]]), I, X.n + J, with_abs=True)
    got = out[torch.as_tensor(I, device="cuda:0"),
              torch.as_tensor(J, device="cuda:0")].cpu().numpy()
    res = {"workload": "cross-set L1 matrix, 10,000 x 20,000 PCFs, counts U{50..500}, "
                       "Exp(1) gaps, N(0,1) values, FP64; per call: plan, pack both sets, "
                       "compute",
           "rows": int(X.n), "cols": int(Y.n), "pairs": pairs, "merge_steps": msteps,
           "ms_per_call": ms, "pairs_per_s": pairs / (ms * 1e-3),
           "merge_steps_per_s": msteps / (ms * 1e-3),
           "parity": dict(pairs=int(len(I)),
                          **err_stats(np.abs(got - ref) / np.maximum(ab, 1e-300)),
                          tolerance=1e-12)}
    if plain_steps_per_s:
        res["vs_plain_merge_steps_per_s"] = res["merge_steps_per_s"] / plain_steps_per_s
    return res


def run_single(steps, warmup):
    """L2 norms of the plain 20,000-PCF set (FP64) by segment iteration: one
    pass over the rows, so HBM-bound; bytes = t and v of every row plus the
    offsets read, one value per PCF written."""
    import torch

    import oracle
    from paper_2404_07183_amd import api, workloads

    o, t, v = workloads.config_plain()
    X = api.PcfSet(o, t, v, device="cuda:0")
    out = torch.empty(X.n, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()
    call = lambda: api.norms(X, 2.0, out=out)
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    # a call takes microseconds: 50 calls captured in a graph and replayed,
    # so that launch gaps do not count
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(stream)
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for _ in range(50):
                call()
    stream.wait_stream(s)
    torch.cuda.synchronize()
    ms = _events_ms(g.replay, steps, stream) / 50
    P = int(o[-1])
    nbytes = P * 16 + (X.n + 1) * 8 + X.n * 8
    ref, ab = oracle.single(oracle.S_NORM, 2.0, 0.0, np.inf, o, t, v, with_abs=True)
    got = out.cpu().numpy()
    return {"workload": "L2 norms of N=20000 PCFs (counts U{50..500}), FP64, one call",
            "pcfs": int(X.n), "rows": P, "ms_per_call": ms,
            "pcfs_per_s": X.n / (ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": nbytes / (ms * 1e-3) / 1e9,
                         "peak": 8000.0, "unit": "GB/s",
                         "frac": nbytes / (ms * 1e-3) / 1e9 / 8000.0,
                         "bytes_per_call": nbytes},
            "parity": dict(pcfs=int(X.n),
                           **err_stats(np.abs(got - ref) / np.maximum(np.sqrt(ab), 1e-300)),
                           tolerance=1e-12)}


def run_reduce(steps, warmup):
    """Mean of the plain 20,000-PCF set (FP64) as one group: a binary tree of
    15 levels, each reading and writing about every row once (continuous
    times share no breakpoints), then the root's rows. Algorithmic bytes:
    per level, t and v of every input row read and of every output row
    written; the root read twice (count, fill) and written once. The time is
    the whole api.reduce call, host round trip for the output size included.
    Also the std of 1,000 groups of 20 PCFs."""
    import torch

    from paper_2404_07183_amd import api, workloads

    o, t, v = workloads.config_plain()
    X = api.PcfSet(o, t, v, device="cuda:0")
    ws = api.Workspace(device="cuda:0")
    stream = torch.cuda.current_stream()
    res = {}
    for name, op, groups in (("mean_one_group", "mean", None),
                             ("std_1000_groups_of_20", "std", np.arange(0, X.n + 1, 20))):
        call = lambda: api.reduce(X, op, groups, workspace=ws)
        for _ in range(warmup):
            out = call()
        torch.cuda.synchronize()
        ms = _events_ms(call, steps, stream)
        res[name] = {"ms_per_call": ms, "out_rows": int(out.offsets_host[-1])}
    P = int(o[-1])
    levels = int(np.ceil(np.log2(X.n)))
    root = res["mean_one_group"]["out_rows"]
    nbytes = levels * 2 * P * 16 + 3 * root * 16
    ms = res["mean_one_group"]["ms_per_call"]
    # parity at sampled times: the tree's mean against NumPy's, within the
    # rounding of a 15-level sum
    out = api.reduce(X, "mean", workspace=ws)
    gt, gv = out.t.cpu().numpy(), out.v.cpu().numpy()
    rng = np.random.default_rng(7)
    x = np.sort(rng.uniform(0.0, float(t.max()) * 1.01, 256))
    vals = np.stack([v[o[i]:o[i + 1]][np.searchsorted(t[o[i]:o[i + 1]], x, side="right") - 1]
                     for i in range(X.n)])
    want = vals.mean(0)
    got = gv[np.searchsorted(gt, x, side="right") - 1]
    err = np.abs(got - want) / np.maximum(np.abs(vals).mean(0), 1e-300)
    res.update({"workload": "mean of N=20000 PCFs (counts U{50..500}) as one group, FP64; "
                            "std of 1000 groups of 20",
                "pcfs": int(X.n), "rows": P, "tree_levels": levels,
                "pcfs_per_s": X.n / (ms * 1e-3),
                "roofline": {"bound": "hbm", "achieved": nbytes / (ms * 1e-3) / 1e9,
                             "peak": 8000.0, "unit": "GB/s",
                             "frac": nbytes / (ms * 1e-3) / 1e9 / 8000.0,
                             "bytes_per_call": nbytes},
                "parity": dict(sampled_times=len(x), **err_stats(err), tolerance=1e-13)})
    return res


def run_bounded_weighted(steps, warmup):
    """L1 distances over [2.5, 40) with the weight w(t) = exp(-0.1 t) on the
    plain 20,000-PCF set (FP64): restriction, time warp and the full matrix
    per call (the restricted and warped set is a new set every call, so its
    tile plan is rebuilt too). Parity on 256 sampled pairs against the
    oracle's per-cell sum of H(r) - H(l)."""
    import torch

    import oracle
    from paper_2404_07183_amd import api, workloads

    o, t, v = workloads.config_plain()
    X = api.PcfSet(o, t, v, device="cuda:0")
    out = torch.empty((X.n, X.n), dtype=torch.float64, device="cuda:0")
    ws = api.Workspace(device="cuda:0")
    stream = torch.cuda.current_stream()
    a, b, c = 2.5, 40.0, 0.1
    call = lambda: api.pdist(X, 1.0, bounds=(a, b), weight=("exp", c), out=out, workspace=ws)
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    ms = _events_ms(call, steps, stream)
    rng = np.random.default_rng(11)
    I, J = rng.integers(0, X.n, 256), rng.integers(0, X.n, 256)
    ref, ab = oracle.entries_w(oracle.LP, 1.0, oracle.W_EXP, c, o, t, v, I, J, a=a, b=b,
                               with_abs=True)
    got = out.cpu().numpy()[I, J]
    pairs = X.n * (X.n - 1) / 2
    return {"workload": "L1 over [2.5, 40) with weight exp(-0.1 t), N=20000 PCFs (counts "
                        "U{50..500}), FP64; restriction + time warp + full matrix per call",
            "ms_per_call": ms, "pairs_per_s": pairs / (ms * 1e-3),
            "parity": dict(pairs=256, **err_stats(np.abs(got - ref) / np.maximum(ab, 1e-300)),
                           tolerance=1e-12)}


def run_general_p(steps, warmup):
    """d_p^p matrices of the plain 20,000-PCF set for p = 3 (squaring),
    p = 3.5 (squaring and a square root) and p = 2.7 (FP64: the 2^(p log2 x)
    series; FP32: the hardware base-2 log and exp), FP64 and FP32; tile plan
    and packed records reused between calls, as in the headline. Parity on
    256 sampled pairs against the oracle (FP32: on the rounded inputs)."""
    import torch

    import oracle
    from paper_2404_07183_amd import api, workloads

    res = {"workload": "d_p^p matrices, N=20000 PCFs (counts U{50..500}), p = 3, 3.5, 2.7"}
    rng = np.random.default_rng(12)
    for dt, name in ((np.float64, "f64"), (np.float32, "f32")):
        o, t, v = workloads.config_plain(dtype=dt)
        X = api.PcfSet(o, t, v, device="cuda:0")
        out = torch.empty((X.n, X.n), dtype=X.dtype, device="cuda:0")
        ws = api.Workspace(device="cuda:0")
        stream = torch.cuda.current_stream()
        I, J = rng.integers(0, X.n, 256), rng.integers(0, X.n, 256)
        for p in (3.0, 3.5, 2.7):
            api.pdist(X, p, power=True, out=out, workspace=ws)
            for _ in range(warmup):
                api.pdist(X, p, power=True, out=out, workspace=ws, packed=True)
            torch.cuda.synchronize()
            ms = _events_ms(lambda: api.pdist(X, p, power=True, out=out, workspace=ws,
                                              packed=True), steps, stream)
            ref, ab = oracle.entries(oracle.LP_POW, p, o, t.astype(np.float64),
                                     v.astype(np.float64), I, J, with_abs=True)
            got = out.cpu().numpy().astype(np.float64)[I, J]
            res["p%g_%s" % (p, name)] = {
                "ms_per_call": ms,
                "max_error_over_scale": float(np.max(np.abs(got - ref) / np.maximum(ab, 1e-300)))}
    return res


def run_grad(steps, warmup, plain_steps_per_s=None):
    """Forward + adjoint of L = sum W_ij d_2(f_i,f_j)^2 + sum U_ij <f_i,f_j>,
    N = 4,096 PCFs, FP64 (two forward matrices, two adjoint passes)."""
    import torch

    from paper_2404_07183_amd import api, workloads

    o, t, v, W, U = workloads.config_grad()
    X = api.PcfSet(o, t, v, device="cuda:0")
    Wt = torch.as_tensor(W, device="cuda:0")
    Ut = torch.as_tensor(U, device="cuda:0")
    tt = X.t.clone().requires_grad_(True)
    vv = X.v.clone().requires_grad_(True)
    stream = torch.cuda.current_stream()

    def step():
        tt.grad = None
        vv.grad = None
        M1 = api.pairwise_matrix(X, tt, vv, api.PCF_LP_POW, 2.0)
        M2 = api.pairwise_matrix(X, tt, vv, api.PCF_GRAM)
        L = (Wt * M1).sum() + (Ut * M2).sum()
        L.backward()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ms = _events_ms(step, steps, stream)
    N = X.n
    n = np.diff(o).astype(np.float64)
    fwd_steps = 2 * (N - 1) * np.sum(n - 1) + 2 * np.sum(n - 1)  # two matrices (+Gram diagonal)
    pairs = N * (N + 1) / 2
    res = {"workload": "loss sum W d_2^2 + sum U <,>, N=4096, counts U{20..300}, FP64; forward "
                       "of both matrices and their adjoints (dL/dt, dL/dv)",
           "pcfs": N, "pairs": pairs, "ms_per_step": ms,
           "fwd_bwd_pairs_per_s": pairs / (ms * 1e-3),
           "merge_steps_per_s_fwd_plus_bwd": 2 * fwd_steps / (ms * 1e-3)}
    if plain_steps_per_s:
        res["vs_plain_merge_steps_per_s"] = res["merge_steps_per_s_fwd_plus_bwd"] / plain_steps_per_s
    # the adjoint kernels alone (plan reused, records packed; each call also
    # clears the two gradient arrays): d_2^2 with weights 2W (the upper
    # triangle's pairs once, each with G_ij + G_ji) and Gram with 2U
    one_steps = (N - 1) * np.sum(n - 1)          # pairs i < j
    adj = {}
    for name, kind, p, G, k_ops, extra in (("l2sq", api.PCF_LP_POW, 2.0, Wt, ADJ_OPS["l2sq"], 0),
                                           ("gram", api.PCF_GRAM, 0.0, Ut, ADJ_OPS["gram"],
                                            np.sum(n - 1))):
        ws = api.Workspace(device="cuda:0")
        api.pairwise_backward(X, kind, p, G, workspace=ws)
        k_ms = _events_ms(lambda: api.pairwise_backward(X, kind, p, G, workspace=ws,
                                                        packed=True), steps, stream)
        # the same call with PCF_DETERMINISTIC (the two bound passes, integer
        # sums in HBM, the conversion pass)
        d_ms = _events_ms(lambda: api.pairwise_backward(X, kind, p, G, workspace=ws,
                                                        packed=True, deterministic=True),
                          steps, stream)
        ops = (one_steps + extra) * k_ops
        adj[name] = {"kernel": "pairwise_adjoint_tiles<%s>" % name, "kernel_ms": k_ms,
                     "call_ms_deterministic": d_ms,
                     "merge_steps": one_steps + extra, "ops_per_step": k_ops,
                     "achieved": ops / (k_ms * 1e-3) / 1e12,
                     "frac": ops / (k_ms * 1e-3) / PEAK_FP64_LANE_OPS}
    # the same adjoint calls on the set rounded to FP32 (merge and terms in
    # FP32, fixed-point tile sums, FP32 atomics)
    t32 = t.astype(np.float32)
    for i in range(N):  # (times kept strictly increasing after rounding)
        for k in range(o[i] + 1, o[i + 1]):
            if t32[k] <= t32[k - 1]:
                t32[k] = np.nextafter(t32[k - 1], np.float32(np.inf))
    X32 = api.PcfSet(o, t32, v.astype(np.float32), device="cuda:0")
    for name, kind, p, G in (("l2sq", api.PCF_LP_POW, 2.0, Wt), ("gram", api.PCF_GRAM, 0.0, Ut)):
        ws = api.Workspace(device="cuda:0")
        api.pairwise_backward(X32, kind, p, G, workspace=ws)
        adj[name]["call_ms_fp32"] = _events_ms(
            lambda: api.pairwise_backward(X32, kind, p, G, workspace=ws, packed=True), steps,
            stream)
    tot_ops = sum(a["merge_steps"] * a["ops_per_step"] for a in adj.values())
    tot_ms = sum(a["kernel_ms"] for a in adj.values())
    res["roofline"] = {"bound": "alu", "achieved": tot_ops / (tot_ms * 1e-3) / 1e12,
                       "peak": PEAK_FP64_LANE_OPS / 1e12, "unit": "TOP/s",
                       "frac": tot_ops / (tot_ms * 1e-3) / PEAK_FP64_LANE_OPS,
                       "kernel": "pairwise_adjoint_tiles (both matrices)",
                       "kernel_ms": tot_ms, "per_kernel": adj}
    if plain_steps_per_s:
        res["adjoint_vs_plain_merge_steps_per_s"] = (
            sum(a["merge_steps"] for a in adj.values()) / (tot_ms * 1e-3) / plain_steps_per_s)
    # parity: the full gradients of four PCFs against the oracle's adjoint
    # of the same loss (only the pairs that involve each PCF matter to it)
    import oracle
    step()
    torch.cuda.synchronize()
    gt, gv = tt.grad.cpu().numpy(), vv.grad.cpu().numpy()
    errs = []
    for i in (0, 1, 2047, N - 1):
        Wi = np.zeros_like(W)
        Ui = np.zeros_like(U)
        Wi[i, :], Wi[:, i] = W[i, :], W[:, i]
        Ui[i, :], Ui[:, i] = U[i, :], U[:, i]
        rt1, rv1 = oracle.backward(oracle.LP_POW, 2.0, o, t, v, Wi)
        rt2, rv2 = oracle.backward(oracle.GRAM, 0.0, o, t, v, Ui)
        a, b = o[i], o[i + 1]
        for g, r in ((gt[a:b], rt1[a:b] + rt2[a:b]), (gv[a:b], rv1[a:b] + rv2[a:b])):
            errs.append(np.abs(g - r) / max(np.max(np.abs(r)), 1e-300))
    res["parity"] = dict(pcfs=4, entries=int(sum(len(e) for e in errs)),
                         **err_stats(np.concatenate(errs)), tolerance=1e-11,
                         reference="oracle adjoint; error over the largest |gradient| of "
                                   "each PCF's t or v")
    return res


def run_small(steps, warmup):
    """The 200-PCF L1 matrix (FP64, counts U{10..100}): per-call latency of a
    whole call (plan, upload, pack, kernel; synchronised after every call),
    of a call that reuses the plan and the packed records, and the oracle's
    single-threaded time for the same matrix on this host (the paper finds
    the CPU ahead at small sizes)."""
    import torch

    import oracle
    from paper_2404_07183_amd import api, workloads

    o, t, v = workloads.config_plain_small()
    X = api.PcfSet(o, t, v, device="cuda:0")
    out = torch.empty((X.n, X.n), dtype=torch.float64, device="cuda:0")
    reps = max(20, steps * 5)

    def per_call_us(fn):
        for _ in range(warmup + 2):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
            torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e6

    full = per_call_us(lambda: api.pdist(X, 1.0, out=out))
    ws = api.Workspace(device="cuda:0")
    api.pdist(X, 1.0, out=out, workspace=ws)
    reuse = per_call_us(lambda: api.pdist(X, 1.0, out=out, workspace=ws, packed=True))
    t0 = time.perf_counter()
    ref = oracle.matrix(oracle.LP, 1.0, o, t, v)
    cpu_us = (time.perf_counter() - t0) * 1e6
    got = out.cpu().numpy()
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
    pairs = X.n * (X.n - 1) / 2
    return {"workload": "L1 matrix of N=200 PCFs, counts U{10..100}, FP64",
            "pairs": pairs, "us_per_call_full": full, "us_per_call_plan_reused": reuse,
            "oracle_single_thread_us_full_matrix": cpu_us,
            "pairs_per_s_full": pairs / (full * 1e-6),
            "parity": dict(entries=int(got.size), **err_stats(err[ref > 0]), tolerance=1e-12)}


def run_strip(args):
    """One GPU's share of the 500,000-PCF stress run: the 62,500 x 500,000
    strip of the L1 matrix (FP32), computed in column chunks into a ring of two
    device buffers, each chunk copied to pinned host memory on a second stream
    while the next one is computed."""
    import torch

    from paper_2404_07183_amd import api, workloads

    t_gen = time.perf_counter()
    o, t, v = workloads.config_strip()
    t_gen = time.perf_counter() - t_gen
    X = api.PcfSet(o, t, v, device="cuda:0")
    N = X.n
    rows = N // 8
    # chunk 0 is the rows x rows diagonal block (a symmetric window: each pair
    # once, written twice); chunks 1.. are rectangles right of it
    cw = rows
    nchunks = min(args.strip_chunks, (N + cw - 1) // cw)
    bufs = [torch.empty((rows, cw), dtype=torch.float32, device="cuda:0") for _ in range(2)]
    host = [torch.empty((rows, cw), dtype=torch.float32, pin_memory=True) for _ in range(2)]
    wss = [api.Workspace(device="cuda:0") for _ in range(2)]
    compute = torch.cuda.current_stream()
    copy = torch.cuda.Stream()
    done = [torch.cuda.Event() for _ in range(2)]
    copied = [torch.cuda.Event() for _ in range(2)]
    # warm-up: plan both buffers' first windows
    api.pdist(X, 1.0, window=(0, rows, 0, cw), out=bufs[0], workspace=wss[0])
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(compute)
    for c in range(nchunks):
        k = c % 2
        c0, c1 = c * cw, min((c + 1) * cw, N)
        if c >= 2:
            compute.wait_event(copied[k])
        out = bufs[k][:, :c1 - c0]
        api.pdist(X, 1.0, window=(0, rows, c0, c1), out=out, workspace=wss[k])
        done[k].record(compute)
        with torch.cuda.stream(copy):
            copy.wait_event(done[k])
            host[k][:, :c1 - c0].copy_(out, non_blocking=True)
            copied[k].record(copy)
    e1.record(compute)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cols = min(nchunks * cw, N)
    # distinct pair integrals computed: rows x cols minus the mirrored half and
    # the diagonal of the rows x rows block
    d = min(rows, cols)
    integrals = rows * cols - d * (d + 1) / 2.0
    return {
        "metric": "PCF pair-integrals/sec (L1, F32, strip)",
        "value": integrals / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1, "steps": nchunks, "warmup": 1, "ms_per_step": ms / nchunks,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "strip of the L1 matrix of 500,000 stable-rank-like PCFs: rows "
                               "0..%d x columns 0..%d, FP32, %d-column chunks streamed to "
                               "pinned host memory" % (rows - 1, cols - 1, cw),
                   "pcfs": N, "rows_in_strip": rows, "columns_done": cols,
                   "generation_s": t_gen},
        "wall_ms": ms,
    }


def calibration_copy():
    """One plain 1 GiB device-to-device copy: a reference for HBM byte counters."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="plain", choices=["plain", "strip"])
    ap.add_argument("--strip-chunks", type=int, default=8,
                    help="column chunks of the strip to compute (8 = all)")
    ap.add_argument("--kind", default="l1", choices=["l1", "l2", "l2sq", "gram"])
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (a reference "
                         "for HBM byte counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and forward+adjoint measurements")
    ap.add_argument("--only", default=None,
                    help="comma-separated extra lines to run alone, without the headline "
                         "(batched, fwd_bwd, cross, single, reduce, bounded_weighted, "
                         "general_p, small)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.only:
        runs = {"batched": lambda k, w: run_batched(k, w), "fwd_bwd": lambda k, w: run_grad(k, w),
                "small": run_small,
                "cross": lambda k, w: run_cross(k, w), "single": run_single,
                "reduce": run_reduce, "bounded_weighted": run_bounded_weighted,
                "general_p": run_general_p}
        names = args.only.split(",")
        bad = [n for n in names if n not in runs]
        if bad:
            ap.error("unknown line(s) for --only: %s" % ", ".join(bad))
        if args.calibration_copy:
            calibration_copy()
        print(json.dumps({n: runs[n](args.steps, args.warmup) for n in names}), flush=True)
        return
    if args.calibration_copy:
        calibration_copy()
    if args.config == "strip":
        print(json.dumps(run_strip(args)), flush=True)
        return
    res = run_plain(args)
    if not args.no_extras:
        plain = res["merge_steps_per_s"]
        res["batched"] = run_batched(max(2, args.steps // 2), 1, plain)
        res["fwd_bwd"] = run_grad(max(2, args.steps // 2), 1, plain)
        res["cross"] = run_cross(max(2, args.steps // 2), 1, plain)
        res["single"] = run_single(max(2, args.steps // 2), 1)
        res["reduce"] = run_reduce(max(2, args.steps // 2), 1)
        res["bounded_weighted"] = run_bounded_weighted(max(2, args.steps // 2), 1)
        res["small"] = run_small(max(2, args.steps // 2), 1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
