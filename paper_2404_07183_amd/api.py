"""PyTorch-facing helpers over the C ABI.

PyTorch provides device memory and the current HIP stream; every step of the
computation runs in ``libpcf.so``. A :class:`PcfSet` holds one ragged CSR set
of PCFs on the GPU (``offsets`` int64, ``t`` and ``v`` FP32 or FP64) plus a
host copy of the offsets, so planning needs no device-to-host copy.
"""
from __future__ import annotations

import ctypes

import math

import numpy as np
import torch

from . import _lib
from ._lib import (PCF_F32, PCF_F64, PCF_GRAM, PCF_LP, PCF_LP_POW,
                   PCF_DETERMINISTIC, PCF_RECORDS_PACKED, PCF_REUSE_PLAN, PCF_UPPER_ONLY,
                   PCF_VALIDATE, PCF_WEIGHT_EXP, PCF_WEIGHT_POW, PCF_REDUCE_SUM,
                   PCF_REDUCE_MEAN, PCF_REDUCE_MAX, PCF_REDUCE_MIN, PCF_REDUCE_STD, check)

__all__ = ["PcfSet", "Workspace", "pdist", "gram", "cdist", "cross_gram", "pairwise_backward",
           "pairwise_batched", "validate", "pairwise_matrix", "PairwiseMatrix",
           "integrals", "norms", "restrict", "warp", "reduce", "combine",
           "restrict_backward", "warp_backward", "pairwise_terms",
           "autotune", "TuneCache", "workload_signature", "TILE_SHAPES", "PCF_LP",
           "PCF_LP_POW", "PCF_GRAM"]


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class PcfSet:
    """A CSR set of PCFs resident on one GPU."""

    def __init__(self, offsets, t, v, device="cuda"):
        if isinstance(offsets, torch.Tensor):
            offsets = offsets.detach().cpu().numpy()
        self.offsets_host = np.ascontiguousarray(offsets, dtype=np.int64)
        self.offsets = torch.as_tensor(self.offsets_host, device=device)
        self.t = torch.as_tensor(t, device=device).contiguous()
        self.v = torch.as_tensor(v, device=device).contiguous()
        if self.t.dtype != self.v.dtype or self.t.dtype not in (torch.float32, torch.float64):
            raise TypeError("t and v must both be float32 or both float64")
        if self.t.numel() != self.v.numel() or self.t.numel() != int(self.offsets_host[-1]):
            raise ValueError("t, v and offsets disagree on the number of rows")
        self.n = len(self.offsets_host) - 1

    @property
    def dtype(self):
        return self.t.dtype

    def with_values(self, t, v):
        """Same offsets, new (t, v) tensors (e.g. ones that require grad)."""
        new = object.__new__(PcfSet)
        new.offsets_host, new.offsets, new.n = self.offsets_host, self.offsets, self.n
        new.t, new.v = t.contiguous(), v.contiguous()
        return new

    def c_struct(self):
        return _lib.pcf_set(
            self.n, self.offsets.data_ptr(), self.t.data_ptr(), self.v.data_ptr(),
            PCF_F64 if self.t.dtype == torch.float64 else PCF_F32,
            self.offsets_host.ctypes.data)


class Workspace:
    """Device workspace; keeps the tile plan between calls on one set."""

    def __init__(self, nbytes=0, device="cuda"):
        self.buf = None
        self.device = device
        self.planned = None
        self.packed_data = None
        self.ensure(nbytes)

    def ensure(self, nbytes):
        nbytes = int(max(nbytes, 256))
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.planned = None
            self.packed_data = None
        return self

    @property
    def ptr(self):
        return self.buf.data_ptr()

    @property
    def nbytes(self):
        return self.buf.numel()


def _window(window):
    if window is None:
        return None
    r0, r1, c0, c1 = (int(x) for x in window)
    return _lib.pcf_window(r0, r1, c0, c1)


def _flags(upper_only, validate, reuse, shape=None):
    f = ((PCF_UPPER_ONLY if upper_only else 0) | (PCF_VALIDATE if validate else 0)
         | (PCF_REUSE_PLAN if reuse else 0))
    if shape is not None:
        max_block, budget_div = shape
        f |= ((int(max_block) & 63) << 8) | ((int(budget_div) & 15) << 16)
    return f


def _check_out(out, X, oshape):
    """A caller's output matrix: the input's dtype and device, row-major,
    at least ``oshape`` (the library writes rows of ``oshape[1]`` entries at
    stride ``out.stride(0)``)."""
    if out.dtype != X.dtype or out.dim() != 2 or out.stride(1) != 1:
        raise ValueError("out must be a row-major 2-D tensor of the input dtype")
    if out.device != X.t.device:
        raise ValueError("out must be on the device of the set (%s), not %s"
                         % (X.t.device, out.device))
    if out.shape[0] < oshape[0] or out.shape[1] < oshape[1]:
        raise ValueError("out has shape %s; the result needs %s"
                         % (tuple(out.shape), tuple(oshape)))


def _forward(X, kind, p, window, out, upper_only, validate, workspace, stream,
             packed=False, shape=None):
    Xc = X.c_struct()
    win = _window(window)
    if window is None:
        oshape = (X.n, X.n)
    else:
        oshape = (window[1] - window[0], window[3] - window[2])
    if out is None:
        out = torch.zeros(oshape, dtype=X.dtype, device=X.t.device)
    _check_out(out, X, oshape)
    ldo = out.stride(0) if out.shape[0] > 1 else max(out.shape[1], 1)
    # the plan depends on the record size (dtype) and on the plan type
    # (forward here; the adjoint's plan has other blocks)
    key = ("fwd", kind, X.dtype, X.n, id(X.offsets_host), window, upper_only, shape, ldo)
    ws = workspace if workspace is not None else Workspace(device=X.t.device)
    reuse = ws.planned == key
    if not reuse:
        ws.ensure(_lib.pcf_workspace_bytes(Xc, kind, win, 0))
    flags = _flags(upper_only, validate, reuse, shape)
    if packed:
        if not reuse or ws.packed_data != (X.t.data_ptr(), X.v.data_ptr()):
            raise ValueError("packed=True needs an earlier call on the same set, "
                             "data and workspace")
        flags |= PCF_RECORDS_PACKED
    if kind == PCF_GRAM:
        st = _lib.pcf_gram(Xc, out.data_ptr(), ldo, win, ws.ptr, ws.nbytes, flags,
                           _stream_handle(stream))
    else:
        st = _lib.pcf_pairwise_lp(Xc, kind, float(p), out.data_ptr(), ldo, win, ws.ptr,
                                  ws.nbytes, flags, _stream_handle(stream))
    check(st)
    ws.planned = key
    ws.planned_ref = X.offsets_host  # keeps id() in the key unique
    ws.packed_data = (X.t.data_ptr(), X.v.data_ptr())
    return out


def pdist(X, p=1.0, *, power=False, window=None, out=None, upper_only=False,
          validate=False, workspace=None, stream=None, packed=False, shape=None,
          bounds=None, weight=None):
    """L_p distance matrix (``power=True``: d_p^p) of the PCFs in ``X``;
    ``bounds=(a, b)``: of the integrals over [a, b) (Section 2.2);
    ``weight=("exp", c)`` or ``("pow", c)``: with the time weight
    w(t) = exp(-c t) or t^c (the weighted L_p distance of Section 2.2).

    ``packed=True`` skips re-packing the breakpoint records: only valid when
    ``workspace`` served the previous call on this very set and data."""
    X = _transform(X, bounds, weight, stream)
    return _forward(X, PCF_LP_POW if power else PCF_LP, p, window, out, upper_only,
                    validate, workspace, stream, packed, shape)


def gram(X, *, window=None, out=None, upper_only=False, validate=False,
         workspace=None, stream=None, packed=False, shape=None, bounds=None,
         weight=None):
    """L2 Gram matrix of the PCFs in ``X`` (``bounds=(a, b)``: over [a, b);
    ``weight``: the weighted inner product, as in ``pdist``)."""
    X = _transform(X, bounds, weight, stream)
    return _forward(X, PCF_GRAM, 0.0, window, out, upper_only, validate, workspace,
                    stream, packed, shape)


def pairwise_terms(X, terms, root=None, *, window=None, out=None, upper_only=False,
                   workspace=None, stream=None):
    """The matrix r(sum_m coef_m I_m(f_i, f_j)) of a time-dependent combination
    h(a, b, t) = sum_m coef_m h0_m(a, b) w_m(t) (Section 3: H(a, b, r) -
    H(a, b, l) per rectangle with H = sum_m coef_m h0_m W_m). ``terms``: a list
    of ``(h0, p, weight, coef)`` with h0 ``"lp"`` (|a - b|^p) or ``"gram"``
    (a b, p ignored) and weight None, ``("exp", c)`` or ``("pow", c)``.
    ``root``: q for r(x) = x^(1/q), or None. Synchronises once per weighted
    term."""
    Xc = X.c_struct()
    win = _window(window)
    oshape = (X.n, X.n) if window is None else (window[1] - window[0], window[3] - window[2])
    if out is None:
        out = torch.zeros(oshape, dtype=X.dtype, device=X.t.device)
    _check_out(out, X, oshape)
    ldo = out.stride(0) if out.shape[0] > 1 else max(out.shape[1], 1)
    ct = []
    for h0, p, weight, coef in terms:
        kind = {"lp": PCF_LP_POW, "gram": PCF_GRAM}[h0]
        wk, c = (0, 0.0) if weight is None else (_WEIGHTS.get(weight[0], weight[0]), weight[1])
        ct.append(_lib.pcf_term(int(kind), float(p) if kind == PCF_LP_POW else 0.0, int(wk),
                                float(c), float(coef)))
    flags = PCF_UPPER_ONLY if upper_only else 0
    ws = workspace if workspace is not None else Workspace(device=X.t.device)
    ws.ensure(_lib.pcf_terms_workspace_bytes(Xc, win, flags))
    ws.planned = None
    ws.packed_data = None
    check(_lib.pcf_pairwise_terms(Xc, ct, float(root) if root else 0.0, out.data_ptr(), ldo,
                                  win, ws.ptr, ws.nbytes, flags, _stream_handle(stream)))
    return out


def _cross(X, Y, kind, p, out, validate, workspace, stream, shape=None):
    if X.dtype != Y.dtype:
        raise ValueError("X and Y must share their dtype")
    Xc, Yc = X.c_struct(), Y.c_struct()
    if Y.t.device != X.t.device:
        raise ValueError("X and Y must be on one device")
    if out is None:
        out = torch.zeros((X.n, Y.n), dtype=X.dtype, device=X.t.device)
    _check_out(out, X, (X.n, Y.n))
    ldo = out.stride(0) if out.shape[0] > 1 else max(out.shape[1], 1)
    ws = workspace if workspace is not None else Workspace(device=X.t.device)
    ws.ensure(_lib.pcf_cross_workspace_bytes(Xc, Yc))
    flags = _flags(False, validate, False, shape)
    check(_lib.pcf_cross(Xc, Yc, kind, float(p), out.data_ptr(), ldo, ws.ptr, ws.nbytes,
                         flags, _stream_handle(stream)))
    ws.planned = None  # the cross plan is never reused
    ws.packed_data = None
    return out


def cdist(X, Y, p=1.0, *, power=False, out=None, validate=False, workspace=None,
          stream=None, shape=None, bounds=None, weight=None):
    """L_p distances (``power=True``: d_p^p) between the PCFs of ``X`` (rows)
    and those of ``Y`` (columns); ``bounds`` and ``weight`` as in ``pdist``."""
    X, Y = _transform(X, bounds, weight, stream), _transform(Y, bounds, weight, stream)
    return _cross(X, Y, PCF_LP_POW if power else PCF_LP, p, out, validate, workspace,
                  stream, shape)


def cross_gram(X, Y, *, out=None, validate=False, workspace=None, stream=None,
               shape=None, bounds=None, weight=None):
    """L2 inner products between the PCFs of ``X`` (rows) and ``Y`` (columns);
    ``bounds`` and ``weight`` as in ``pdist``."""
    X, Y = _transform(X, bounds, weight, stream), _transform(Y, bounds, weight, stream)
    return _cross(X, Y, PCF_GRAM, 0.0, out, validate, workspace, stream, shape)


def restrict(X, a, b, stream=None):
    """The PCFs of ``X`` times the indicator of [a, b) (a new set on the same
    device): any matrix of the result is the matrix of integrals over
    [a, b) (Section 2.2). ``b`` may be ``inf``. Synchronises the stream
    once (the output size is read back), so it cannot be graph-captured."""
    Xc = X.c_struct()
    off_h = np.empty(X.n + 1, dtype=np.int64)
    off_d = torch.empty(X.n + 1, dtype=torch.int64, device=X.t.device)
    check(_lib.pcf_restrict_rows(Xc, float(a), float(b), off_d.data_ptr(),
                                 off_h.ctypes.data, _stream_handle(stream)))
    rows = int(off_h[-1])
    t = torch.empty(rows, dtype=X.dtype, device=X.t.device)
    v = torch.empty(rows, dtype=X.dtype, device=X.t.device)
    check(_lib.pcf_restrict(Xc, float(a), float(b), off_d.data_ptr(), t.data_ptr(),
                            v.data_ptr(), _stream_handle(stream)))
    new = object.__new__(PcfSet)
    new.offsets_host, new.offsets, new.n = off_h, off_d, X.n
    new.t, new.v = t, v
    return new


_WEIGHTS = {"exp": PCF_WEIGHT_EXP, "pow": PCF_WEIGHT_POW}


def warp(X, weight, c, stream=None):
    """The PCFs of ``X`` with every breakpoint t carried to W(t), the
    antiderivative of the weight (``"exp"``: w(t) = exp(-c t); ``"pow"``:
    w(t) = t^c). Any matrix of the result is the matrix of the time-weighted
    integrals (Section 3, time-dependent h with antiderivative H).
    Synchronises the stream once (the output size is read back)."""
    wk = _WEIGHTS.get(weight, weight)
    Xc = X.c_struct()
    off_h = np.empty(X.n + 1, dtype=np.int64)
    off_d = torch.empty(X.n + 1, dtype=torch.int64, device=X.t.device)
    check(_lib.pcf_warp_rows(Xc, int(wk), float(c), off_d.data_ptr(), off_h.ctypes.data,
                             _stream_handle(stream)))
    rows = int(off_h[-1])
    t = torch.empty(rows, dtype=X.dtype, device=X.t.device)
    v = torch.empty(rows, dtype=X.dtype, device=X.t.device)
    check(_lib.pcf_warp(Xc, int(wk), float(c), off_d.data_ptr(), t.data_ptr(), v.data_ptr(),
                        _stream_handle(stream)))
    new = object.__new__(PcfSet)
    new.offsets_host, new.offsets, new.n = off_h, off_d, X.n
    new.t, new.v = t, v
    return new


def restrict_backward(X, a, b, Y, grad_t, grad_v, stream=None):
    """dL/dt, dL/dv of ``X``'s rows (FP64) from those of ``Y = restrict(X, a,
    b)``'s rows: kept rows pass theirs on, the row holding ``a`` receives the
    value gradient of Y's row at ``a``, all else is 0 (see pcf.h)."""
    gt = torch.empty(X.t.shape[0], dtype=torch.float64, device=X.t.device)
    gv = torch.empty_like(gt)
    grad_t = grad_t.to(torch.float64).contiguous()
    grad_v = grad_v.to(torch.float64).contiguous()
    check(_lib.pcf_restrict_backward(X.c_struct(), float(a), float(b), Y.offsets.data_ptr(),
                                     grad_t.data_ptr(), grad_v.data_ptr(), gt.data_ptr(),
                                     gv.data_ptr(), _stream_handle(stream)))
    return gt, gv


def warp_backward(X, weight, c, Y, grad_t, grad_v, stream=None):
    """dL/dt, dL/dv of ``X``'s rows (FP64) from those of ``Y = warp(X,
    weight, c)``'s rows: dL/dt_k = dL/dtau_k * w(t_k) (see pcf.h)."""
    wk = _WEIGHTS.get(weight, weight)
    gt = torch.empty(X.t.shape[0], dtype=torch.float64, device=X.t.device)
    gv = torch.empty_like(gt)
    grad_t = grad_t.to(torch.float64).contiguous()
    grad_v = grad_v.to(torch.float64).contiguous()
    check(_lib.pcf_warp_backward(X.c_struct(), int(wk), float(c), Y.offsets.data_ptr(),
                                 grad_t.data_ptr(), grad_v.data_ptr(), gt.data_ptr(),
                                 gv.data_ptr(), _stream_handle(stream)))
    return gt, gv


_REDUCE_OPS = {"sum": PCF_REDUCE_SUM, "mean": PCF_REDUCE_MEAN, "max": PCF_REDUCE_MAX,
               "min": PCF_REDUCE_MIN, "std": PCF_REDUCE_STD}


def reduce(X, op="mean", groups=None, workspace=None, stream=None):
    """Reduce groups of the PCFs in ``X`` (Section 2.1 reductions, Section 4
    reduction trees): ``op`` in sum, mean, max, min, std (sample, 1/(m-1)).
    ``groups``: B+1 offsets into the set's PCFs (default: one group of all).
    Returns a set of B PCFs. Synchronises the stream once (the output size
    is read back)."""
    opc = _REDUCE_OPS.get(op, op)
    g = np.ascontiguousarray([0, X.n] if groups is None else groups, dtype=np.int64)
    B = len(g) - 1
    Xc = X.c_struct()
    ws = workspace if workspace is not None else Workspace(device=X.t.device)
    ws.ensure(_lib.pcf_reduce_workspace_bytes(Xc, B, g.ctypes.data, int(opc)))
    off_h = np.empty(B + 1, dtype=np.int64)
    off_d = torch.empty(B + 1, dtype=torch.int64, device=X.t.device)
    check(_lib.pcf_reduce_rows(Xc, B, g.ctypes.data, int(opc), ws.ptr, ws.nbytes,
                               off_d.data_ptr(), off_h.ctypes.data, _stream_handle(stream)))
    rows = int(off_h[-1])
    t = torch.empty(rows, dtype=X.dtype, device=X.t.device)
    v = torch.empty(rows, dtype=X.dtype, device=X.t.device)
    check(_lib.pcf_reduce(Xc, B, g.ctypes.data, int(opc), ws.ptr, ws.nbytes, off_d.data_ptr(),
                          t.data_ptr(), v.data_ptr(), _stream_handle(stream)))
    ws.planned = None
    ws.packed_data = None
    new = object.__new__(PcfSet)
    new.offsets_host, new.offsets, new.n = off_h, off_d, B
    new.t, new.v = t, v
    return new


_COMBINE_OPS = {"sum": 0, "sub": 1, "mul": 2, "max": 3, "min": 4, "sqdiff": 5}


def combine(X, Y, op="sum", workspace=None, stream=None):
    """The induced combination h_*(x_i, y_i) of two sets index by index
    (Section 2.1): ``op`` in sum, sub, mul, max, min, sqdiff. Returns a set
    of n PCFs. Synchronises the stream once (the output size is read back)."""
    opc = _COMBINE_OPS.get(op, op)
    Xc, Yc = X.c_struct(), Y.c_struct()
    ws = workspace if workspace is not None else Workspace(device=X.t.device)
    ws.ensure(_lib.pcf_combine_workspace_bytes(Xc, Yc, int(opc)))
    off_h = np.empty(X.n + 1, dtype=np.int64)
    off_d = torch.empty(X.n + 1, dtype=torch.int64, device=X.t.device)
    check(_lib.pcf_combine_rows(Xc, Yc, int(opc), ws.ptr, ws.nbytes, off_d.data_ptr(),
                                off_h.ctypes.data, _stream_handle(stream)))
    rows = int(off_h[-1])
    t = torch.empty(rows, dtype=X.dtype, device=X.t.device)
    v = torch.empty(rows, dtype=X.dtype, device=X.t.device)
    check(_lib.pcf_combine(Xc, Yc, int(opc), ws.ptr, ws.nbytes, off_d.data_ptr(), t.data_ptr(),
                           v.data_ptr(), _stream_handle(stream)))
    ws.planned = None
    ws.packed_data = None
    new = object.__new__(PcfSet)
    new.offsets_host, new.offsets, new.n = off_h, off_d, X.n
    new.t, new.v = t, v
    return new


def _transform(X, bounds, weight, stream):
    """Restriction to ``bounds``, then the time warp of ``weight``."""
    if bounds is not None:
        X = restrict(X, *bounds, stream=stream)
    if weight is not None:
        X = warp(X, *weight, stream=stream)
    return X


def _single(X, kind, p, a, b, out, stream):
    if out is None:
        out = torch.empty(X.n, dtype=X.dtype, device=X.t.device)
    if out.dtype != X.dtype or out.numel() != X.n or not out.is_contiguous():
        raise ValueError("out must be a contiguous vector of n entries of the input dtype")
    check(_lib.pcf_single(X.c_struct(), kind, float(p), float(a), float(b),
                          out.data_ptr(), _stream_handle(stream)))
    return out


def integrals(X, a=0.0, b=math.inf, *, out=None, stream=None):
    """int_a^b f_i for every PCF of ``X`` (Section 3.2)."""
    return _single(X, _lib.PCF_INTEGRAL, 1.0, a, b, out, stream)


def norms(X, p=2.0, a=0.0, b=math.inf, *, power=False, out=None, stream=None):
    """L_p norms (``power=True``: int |f_i|^p; ``p=inf``: sup |f_i|) of the
    PCFs of ``X`` over [a, b)."""
    if p == math.inf:
        return _single(X, _lib.PCF_NORM_INF, 0.0, a, b, out, stream)
    return _single(X, _lib.PCF_NORM_POW if power else _lib.PCF_NORM, p, a, b, out, stream)


def pairwise_backward(X, kind, p, grad_out, fwd_out=None, workspace=None, stream=None,
                      packed=False, deterministic=False):
    """(dL/dt, dL/dv) for a loss with dL/dF = grad_out (n x n, taken in
    FP64), in the set's dtype (FP32 or FP64; FP32 sets merge in FP32 with the
    gradient sums in 64-bit fixed point, then FP32 atomics into the result).
    A ``workspace`` that served the previous backward call on the same set
    keeps its plan; ``packed=True`` as in ``pdist``. ``deterministic=True``
    sums the gradients in 64-bit fixed point at the set's scales: the same
    bits on every run (PCF_DETERMINISTIC)."""
    Xc = X.c_struct()
    grad_out = grad_out.to(torch.float64).contiguous()
    if grad_out.shape != (X.n, X.n) or grad_out.device != X.t.device:
        raise ValueError("grad_out must be an n x n tensor on the set's device")
    gt = torch.empty_like(X.t)
    gv = torch.empty_like(X.v)
    key = ("bwd", kind, X.dtype, X.n, id(X.offsets_host))
    ws = workspace if workspace is not None else Workspace(device=X.t.device)
    reuse = ws.planned == key
    if not reuse:
        ws.ensure(_lib.pcf_workspace_bytes(Xc, kind, None, 1))
    flags = PCF_REUSE_PLAN if reuse else 0
    if packed:
        if not reuse or ws.packed_data != (X.t.data_ptr(), X.v.data_ptr()):
            raise ValueError("packed=True needs an earlier call on the same set, "
                             "data and workspace")
        flags |= PCF_RECORDS_PACKED
    if deterministic:
        flags |= PCF_DETERMINISTIC
    fptr, ldf = (fwd_out.data_ptr(), fwd_out.stride(0)) if fwd_out is not None else (None, 0)
    st = _lib.pcf_pairwise_backward(Xc, kind, float(p), grad_out.data_ptr(),
                                    grad_out.stride(0), fptr, ldf, gt.data_ptr(),
                                    gv.data_ptr(), ws.ptr, ws.nbytes, flags,
                                    _stream_handle(stream))
    check(st)
    ws.planned = key
    ws.planned_ref = X.offsets_host
    ws.packed_data = (X.t.data_ptr(), X.v.data_ptr())
    return gt, gv


def pairwise_batched(set_offsets, X, kind=PCF_LP, p=1.0, *, out=None, workspace=None,
                     upper_only=False, validate=False, stream=None, shape=None,
                     bounds=None, weight=None, packed=False):
    """Independent full matrices of the problems ``set_offsets`` cuts ``X``
    into, in one launch. Returns ``(out_flat, out_offsets)``: problem b's
    s_b x s_b matrix is ``out_flat[out_offsets[b]:][:s_b*s_b]``.
    ``bounds`` and ``weight`` as in ``pdist`` (the set is transformed first;
    PCF indices are kept). ``packed=True`` as in ``pdist``."""
    X = _transform(X, bounds, weight, stream)
    so = np.ascontiguousarray(set_offsets, dtype=np.int64)
    B = len(so) - 1
    sizes = np.diff(so)
    oo = np.zeros(B, dtype=np.int64)
    if B > 1:
        oo[1:] = np.cumsum(sizes[:-1] ** 2)
    total = int((sizes ** 2).sum())
    if out is None:
        out = torch.zeros(total, dtype=X.dtype, device=X.t.device)
    if out.dtype != X.dtype or not out.is_contiguous() or out.device != X.t.device:
        raise ValueError("out must be a contiguous tensor of the set's dtype and device")
    if out.numel() < total:
        raise ValueError("out holds %d entries; the matrices need %d" % (out.numel(), total))
    Xc = X.c_struct()
    key = ("batched", kind, X.dtype, X.n, id(X.offsets_host), so.tobytes(), upper_only,
           shape)
    ws = workspace if workspace is not None else Workspace(device=X.t.device)
    reuse = ws.planned == key
    if not reuse:
        ws.ensure(_lib.pcf_batched_workspace_bytes(B, so.ctypes.data, Xc))
    flags = _flags(upper_only, validate, reuse, shape)
    if packed:
        if not reuse or ws.packed_data != (X.t.data_ptr(), X.v.data_ptr()):
            raise ValueError("packed=True needs an earlier call on the same set, "
                             "data and workspace")
        flags |= PCF_RECORDS_PACKED
    st = _lib.pcf_pairwise_batched(B, so.ctypes.data, Xc, kind, float(p), out.data_ptr(),
                                   oo.ctypes.data, ws.ptr, ws.nbytes, flags,
                                   _stream_handle(stream))
    check(st)
    ws.planned = key
    ws.planned_ref = X.offsets_host
    ws.packed_data = (X.t.data_ptr(), X.v.data_ptr())
    return out, oo


# Tile shapes the autotuner tries: (most PCFs per block, block budget divisor).
TILE_SHAPES = [(32, 2), (16, 2), (32, 3), (24, 2), (8, 2), (32, 4)]
_TUNED = {}


def _bucket(x):
    """log2 bucket of a positive size (0 for x <= 1)."""
    return int(math.floor(math.log2(x))) if x > 1 else 0


def workload_signature(X, kind, p=0.0, set_offsets=None):
    """A tuning key that groups similar workloads: dtype, kind (and for L_p
    whether p is 1, 2 or general), and log2 buckets of the set size, of the
    mean and of the largest row count per PCF; for a batch (``set_offsets``)
    the number of problems and the bucket of their mean size instead of the
    set size. Workloads in one bucket share a tuned tile shape."""
    n = np.diff(X.offsets_host)
    mean_rows = float(n.mean()) if len(n) else 0.0
    pk = "gram" if kind == PCF_GRAM else ("p1" if p == 1.0 else ("p2" if p == 2.0 else "p"))
    if kind == PCF_LP_POW:
        pk += "pow"
    sig = ["f64" if X.dtype == torch.float64 else "f32", pk,
           "rows%d" % _bucket(mean_rows), "max%d" % _bucket(int(n.max()) if len(n) else 0)]
    if set_offsets is None:
        sig.append("n%d" % _bucket(X.n))
    else:
        sizes = np.diff(np.asarray(set_offsets, dtype=np.int64))
        sig += ["b%d" % _bucket(len(sizes)), "s%d" % _bucket(float(sizes.mean()) if len(sizes) else 0)]
    return "/".join(sig)


class TuneCache:
    """Tuned tile shapes kept in a JSON file across processes.

    Entries are keyed by the tuning key together with the device name and a
    digest of the loaded library, so a rebuilt library or another GPU model
    tunes again. The default file is ``$PCF_TUNE_CACHE`` or
    ``~/.cache/paper_2404_07183_amd/tiles.json``. An unreadable file is
    treated as empty; writes replace the file atomically."""

    def __init__(self, path=None):
        import os
        self.path = path or os.environ.get("PCF_TUNE_CACHE") or os.path.join(
            os.path.expanduser("~"), ".cache", "paper_2404_07183_amd", "tiles.json")

    @staticmethod
    def context():
        import hashlib
        import os
        h = hashlib.sha256()
        with open(_lib.LIB_PATH, "rb") as f:
            h.update(f.read())
        dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
        return "%s|%s" % (dev, h.hexdigest()[:16])

    def _load(self):
        import json
        try:
            with open(self.path) as f:
                data = json.load(f)
            return data if isinstance(data, dict) else {}
        except (OSError, ValueError):
            return {}

    def get(self, key, context=None):
        e = self._load().get("%s|%s" % (context or self.context(), key))
        if not e or "shape" not in e:
            return None
        shape = e["shape"]
        return (tuple(shape) if shape is not None else None,
                {(tuple(k) if k is not None else None): ms for k, ms in e.get("times", [])})

    def put(self, key, shape, times, context=None):
        """Stores an entry; returns False (and keeps nothing) when the file
        cannot be written."""
        import json
        import os
        data = self._load()
        data["%s|%s" % (context or self.context(), key)] = {
            "shape": list(shape) if shape is not None else None,
            "times": [[list(k) if k is not None else None, v] for k, v in times.items()]}
        tmp = "%s.tmp%d" % (self.path, os.getpid())
        try:
            d = os.path.dirname(self.path)
            if d:
                os.makedirs(d, exist_ok=True)
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except OSError:
            return False
        return True


def autotune(run, key, shapes=None, reps=3, cache=None):
    """Pick the fastest tile shape for a workload.

    ``run(shape)`` must launch one call with that shape (``None`` = default)
    on the current stream. Every candidate runs once untimed (which also
    builds its plan) and ``reps`` times between HIP events; the shape with the
    smallest mean time wins and is remembered under ``key`` for the process
    and, with ``cache`` (a :class:`TuneCache`, or True for the default file),
    across processes (see :func:`workload_signature` for keys that group
    workloads by size and row-count bucket). Returns ``(shape, {shape: ms})``."""
    if cache is True:
        cache = TuneCache()
    ckey = (key, cache.path if cache else None)
    if ckey in _TUNED:
        return _TUNED[ckey]
    if cache:
        hit = cache.get(str(key))
        if hit is not None:
            _TUNED[ckey] = hit
            return hit
    shapes = shapes or TILE_SHAPES
    stream = torch.cuda.current_stream()
    times = {}
    for shape in shapes:
        run(shape)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run(shape)
        e1.record(stream)
        e1.synchronize()
        times[shape] = e0.elapsed_time(e1) / reps
    best = min(times, key=times.get)
    _TUNED[ckey] = (best, times)
    if cache:
        cache.put(str(key), best, times)
    return _TUNED[ckey]


def validate(X, stream=None):
    """Index of the first PCF that breaks the data contract, or -1."""
    ws = torch.empty(256, dtype=torch.uint8, device=X.t.device)
    return _lib.pcf_validate(X.c_struct(), ws.data_ptr(), 256, _stream_handle(stream))


class PairwiseMatrix(torch.autograd.Function):
    """F(C) as a differentiable function of the breakpoint times and values,
    optionally over a range [a, b) and with a time weight.

    Forward restricts and warps the set (when asked) and runs the pairwise
    kernel; backward runs the adjoint kernel on the transformed set, which
    recomputes every pair's merge (nothing is stored between the two), then
    maps the gradients back through the warp and the restriction."""

    @staticmethod
    def forward(ctx, t, v, X, kind, p, bounds, weight, deterministic=False):
        Xv = X.with_values(t.detach(), v.detach())
        sets = [Xv]
        if bounds is not None:
            sets.append(restrict(sets[-1], bounds[0], bounds[1]))
        if weight is not None:
            sets.append(warp(sets[-1], weight[0], weight[1]))
        out = _forward(sets[-1], kind, p, None, None, False, False, None, None)
        ctx.sets, ctx.kind, ctx.p, ctx.bounds, ctx.weight = sets, kind, p, bounds, weight
        ctx.deterministic = deterministic
        ctx.save_for_backward(out)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (out,) = ctx.saved_tensors
        need_fwd = ctx.kind == PCF_LP and ctx.p != 1.0
        sets = ctx.sets
        gt, gv = pairwise_backward(sets[-1], ctx.kind, ctx.p, grad_out,
                                   out.to(torch.float64) if need_fwd else None,
                                   deterministic=ctx.deterministic)
        k = len(sets) - 1
        if ctx.weight is not None:
            gt, gv = warp_backward(sets[k - 1], ctx.weight[0], ctx.weight[1], sets[k], gt, gv)
            k -= 1
        if ctx.bounds is not None:
            gt, gv = restrict_backward(sets[k - 1], ctx.bounds[0], ctx.bounds[1], sets[k],
                                       gt, gv)
        # (the range and warp maps return FP64; the inputs' dtype comes back)
        dt = sets[0].t.dtype
        return gt.to(dt), gv.to(dt), None, None, None, None, None, None


def pairwise_matrix(X, t, v, kind=PCF_LP, p=1.0, bounds=None, weight=None,
                    deterministic=False):
    """Differentiable F(C) over ``X``'s offsets with times ``t`` and values
    ``v`` (tensors that may require grad); ``bounds=(a, b)`` integrates over
    [a, b), ``weight=("exp"|"pow", c)`` with the time weight (as ``pdist``);
    ``deterministic=True``: bit-identical gradients run to run."""
    return PairwiseMatrix.apply(t, v, X, kind, p, bounds, weight, deterministic)
