"""ctypes binding of ``libpcf.so`` (the C ABI in ``include/pcf.h``).

Argument marshalling only: every computation runs in the HIP library. The
functions keep the C names. Loading fails loudly when the library has not
been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcf.so")

PCF_OK, PCF_EINVAL, PCF_EDATA, PCF_EDEVICE, PCF_ENOMEM, PCF_EUNSUPPORTED = range(6)
PCF_F32, PCF_F64 = 0, 1
PCF_LP, PCF_LP_POW, PCF_GRAM = 0, 1, 2
PCF_UPPER_ONLY, PCF_VALIDATE, PCF_DETERMINISTIC, PCF_REUSE_PLAN = 1, 2, 4, 8
PCF_RECORDS_PACKED = 16
PCF_INTEGRAL, PCF_NORM, PCF_NORM_POW, PCF_NORM_INF = 0, 1, 2, 3
PCF_WEIGHT_EXP, PCF_WEIGHT_POW = 1, 2
PCF_REDUCE_SUM, PCF_REDUCE_MEAN, PCF_REDUCE_MAX, PCF_REDUCE_MIN, PCF_REDUCE_STD = 0, 1, 2, 3, 4
(PCF_COMBINE_SUM, PCF_COMBINE_SUB, PCF_COMBINE_MUL, PCF_COMBINE_MAX, PCF_COMBINE_MIN,
 PCF_COMBINE_SQDIFF) = range(6)

STATUS_NAMES = {0: "PCF_OK", 1: "PCF_EINVAL", 2: "PCF_EDATA", 3: "PCF_EDEVICE",
                4: "PCF_ENOMEM", 5: "PCF_EUNSUPPORTED"}


class pcf_set(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64),
                ("offsets", ctypes.c_void_p),
                ("t", ctypes.c_void_p),
                ("v", ctypes.c_void_p),
                ("dtype", ctypes.c_int),
                ("offsets_host", ctypes.c_void_p)]


class pcf_term(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("p", ctypes.c_double), ("weight", ctypes.c_int),
                ("c", ctypes.c_double), ("coef", ctypes.c_double)]


class pcf_window(ctypes.Structure):
    _fields_ = [("row0", ctypes.c_int64), ("row1", ctypes.c_int64),
                ("col0", ctypes.c_int64), ("col1", ctypes.c_int64)]


class PcfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


_lib = None

# exported symbols and their ctypes signatures
_SIGS = {
    "pcf_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int,
                                           ctypes.POINTER(pcf_window), ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "pcf_pairwise_lp": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int,
                                       ctypes.c_double, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.POINTER(pcf_window), ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_uint32, ctypes.c_void_p]),
    "pcf_pairwise_lp_noalloc": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int,
                                               ctypes.c_double, ctypes.c_void_p,
                                               ctypes.c_int64, ctypes.POINTER(pcf_window),
                                               ctypes.c_uint32, ctypes.c_void_p]),
    "pcf_gram": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_void_p, ctypes.c_int64,
                                ctypes.POINTER(pcf_window), ctypes.c_void_p,
                                ctypes.c_size_t, ctypes.c_uint32, ctypes.c_void_p]),
    "pcf_pairwise_backward": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int,
                                             ctypes.c_double, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_uint32,
                                             ctypes.c_void_p]),
    "pcf_pairwise_batched": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.POINTER(pcf_set), ctypes.c_int,
                                            ctypes.c_double, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_size_t, ctypes.c_uint32,
                                            ctypes.c_void_p]),
    "pcf_batched_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p,
                                                   ctypes.POINTER(pcf_set),
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "pcf_restrict_rows": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_double,
                                         ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "pcf_restrict": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_double,
                                    ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]),
    "pcf_reduce_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int32,
                                                  ctypes.c_void_p, ctypes.c_int,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "pcf_reduce_rows": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "pcf_reduce": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "pcf_combine_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(pcf_set),
                                                   ctypes.POINTER(pcf_set), ctypes.c_int,
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "pcf_combine_rows": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.POINTER(pcf_set),
                                        ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pcf_combine": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.POINTER(pcf_set),
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p]),
    "pcf_warp_rows": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int,
                                     ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "pcf_warp": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int, ctypes.c_double,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p]),
    "pcf_terms_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(pcf_set),
                                                 ctypes.POINTER(pcf_window), ctypes.c_uint32,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "pcf_pairwise_terms": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int32,
                                          ctypes.POINTER(pcf_term), ctypes.c_double,
                                          ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.POINTER(pcf_window), ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_uint32, ctypes.c_void_p]),
    "pcf_restrict_backward": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_double,
                                             ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "pcf_warp_backward": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int,
                                         ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "pcf_single": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "pcf_cross": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.POINTER(pcf_set),
                                 ctypes.c_int, ctypes.c_double, ctypes.c_void_p,
                                 ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t,
                                 ctypes.c_uint32, ctypes.c_void_p]),
    "pcf_cross_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(pcf_set),
                                                 ctypes.POINTER(pcf_set),
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "pcf_validate": (ctypes.c_int, [ctypes.POINTER(pcf_set), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "pcf_plan_inspect": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.POINTER(pcf_window), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.c_void_p, ctypes.c_int64]),
    "pcf_last_error": (ctypes.c_char_p, []),
    "pcf_abi_version": (ctypes.c_int, []),
}


def exported_names():
    return list(_SIGS)


def load():
    """Load ``libpcf.so``; raise if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libpcf.so is not built (expected at %s); run "
                "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def last_error():
    return load().pcf_last_error().decode("utf-8", "replace")


def check(status):
    if status != PCF_OK:
        raise PcfError(status, last_error())
    return status


# Same-name wrappers (the C calls themselves; pointers are ints).
def pcf_workspace_bytes(X, kind, window, backward):
    out = ctypes.c_size_t(0)
    check(load().pcf_workspace_bytes(ctypes.byref(X), kind,
                                     ctypes.byref(window) if window else None,
                                     int(backward), ctypes.byref(out)))
    return out.value


def pcf_pairwise_lp(X, kind, p, out_ptr, ldo, window, ws_ptr, ws_bytes, flags, stream):
    return load().pcf_pairwise_lp(ctypes.byref(X), kind, p, out_ptr, ldo,
                                  ctypes.byref(window) if window else None,
                                  ws_ptr, ws_bytes, flags, stream)


def pcf_gram(X, out_ptr, ldo, window, ws_ptr, ws_bytes, flags, stream):
    return load().pcf_gram(ctypes.byref(X), out_ptr, ldo,
                           ctypes.byref(window) if window else None,
                           ws_ptr, ws_bytes, flags, stream)


def pcf_pairwise_backward(X, kind, p, grad_out_ptr, ldg, fwd_ptr, ldf, gt_ptr, gv_ptr,
                          ws_ptr, ws_bytes, flags, stream):
    return load().pcf_pairwise_backward(ctypes.byref(X), kind, p, grad_out_ptr, ldg,
                                        fwd_ptr, ldf, gt_ptr, gv_ptr, ws_ptr, ws_bytes,
                                        flags, stream)


def pcf_pairwise_batched(B, set_offsets_host_ptr, X, kind, p, out_ptr,
                         out_offsets_host_ptr, ws_ptr, ws_bytes, flags, stream):
    return load().pcf_pairwise_batched(B, set_offsets_host_ptr, ctypes.byref(X), kind, p,
                                       out_ptr, out_offsets_host_ptr, ws_ptr, ws_bytes,
                                       flags, stream)


def pcf_batched_workspace_bytes(B, set_offsets_host_ptr, X):
    out = ctypes.c_size_t(0)
    check(load().pcf_batched_workspace_bytes(B, set_offsets_host_ptr, ctypes.byref(X),
                                             ctypes.byref(out)))
    return out.value


def pcf_restrict_rows(X, a, b, offsets_out_ptr, offsets_out_host_ptr, stream):
    return load().pcf_restrict_rows(ctypes.byref(X), a, b, offsets_out_ptr,
                                    offsets_out_host_ptr, stream)


def pcf_restrict(X, a, b, offsets_out_ptr, t_out_ptr, v_out_ptr, stream):
    return load().pcf_restrict(ctypes.byref(X), a, b, offsets_out_ptr, t_out_ptr,
                               v_out_ptr, stream)


def pcf_reduce_workspace_bytes(X, B, groups_ptr, op):
    out = ctypes.c_size_t(0)
    check(load().pcf_reduce_workspace_bytes(ctypes.byref(X), B, groups_ptr, op,
                                            ctypes.byref(out)))
    return out.value


def pcf_reduce_rows(X, B, groups_ptr, op, ws_ptr, ws_bytes, offsets_out_ptr,
                    offsets_out_host_ptr, stream):
    return load().pcf_reduce_rows(ctypes.byref(X), B, groups_ptr, op, ws_ptr, ws_bytes,
                                  offsets_out_ptr, offsets_out_host_ptr, stream)


def pcf_reduce(X, B, groups_ptr, op, ws_ptr, ws_bytes, offsets_out_ptr, t_out_ptr, v_out_ptr,
               stream):
    return load().pcf_reduce(ctypes.byref(X), B, groups_ptr, op, ws_ptr, ws_bytes,
                             offsets_out_ptr, t_out_ptr, v_out_ptr, stream)


def pcf_combine_workspace_bytes(X, Y, op):
    out = ctypes.c_size_t(0)
    check(load().pcf_combine_workspace_bytes(ctypes.byref(X), ctypes.byref(Y), op,
                                             ctypes.byref(out)))
    return out.value


def pcf_combine_rows(X, Y, op, ws_ptr, ws_bytes, offsets_out_ptr, offsets_out_host_ptr, stream):
    return load().pcf_combine_rows(ctypes.byref(X), ctypes.byref(Y), op, ws_ptr, ws_bytes,
                                   offsets_out_ptr, offsets_out_host_ptr, stream)


def pcf_combine(X, Y, op, ws_ptr, ws_bytes, offsets_out_ptr, t_out_ptr, v_out_ptr, stream):
    return load().pcf_combine(ctypes.byref(X), ctypes.byref(Y), op, ws_ptr, ws_bytes,
                              offsets_out_ptr, t_out_ptr, v_out_ptr, stream)


def pcf_warp_rows(X, weight, c, offsets_out_ptr, offsets_out_host_ptr, stream):
    return load().pcf_warp_rows(ctypes.byref(X), weight, c, offsets_out_ptr,
                                offsets_out_host_ptr, stream)


def pcf_warp(X, weight, c, offsets_out_ptr, t_out_ptr, v_out_ptr, stream):
    return load().pcf_warp(ctypes.byref(X), weight, c, offsets_out_ptr, t_out_ptr,
                           v_out_ptr, stream)


def pcf_terms_workspace_bytes(X, window, flags):
    out = ctypes.c_size_t(0)
    check(load().pcf_terms_workspace_bytes(ctypes.byref(X),
                                           ctypes.byref(window) if window else None, flags,
                                           ctypes.byref(out)))
    return out.value


def pcf_pairwise_terms(X, terms, q, out_ptr, ldo, window, ws_ptr, ws_bytes, flags, stream):
    arr = (pcf_term * len(terms))(*terms)
    return load().pcf_pairwise_terms(ctypes.byref(X), len(terms), arr, q, out_ptr, ldo,
                                     ctypes.byref(window) if window else None, ws_ptr,
                                     ws_bytes, flags, stream)


def pcf_restrict_backward(X, a, b, offsets_y_ptr, gt_y_ptr, gv_y_ptr, gt_x_ptr, gv_x_ptr,
                          stream):
    return load().pcf_restrict_backward(ctypes.byref(X), a, b, offsets_y_ptr, gt_y_ptr,
                                        gv_y_ptr, gt_x_ptr, gv_x_ptr, stream)


def pcf_warp_backward(X, weight, c, offsets_y_ptr, gt_y_ptr, gv_y_ptr, gt_x_ptr, gv_x_ptr,
                      stream):
    return load().pcf_warp_backward(ctypes.byref(X), weight, c, offsets_y_ptr, gt_y_ptr,
                                    gv_y_ptr, gt_x_ptr, gv_x_ptr, stream)


def pcf_single(X, kind, p, a, b, out_ptr, stream):
    return load().pcf_single(ctypes.byref(X), kind, p, a, b, out_ptr, stream)


def pcf_cross(X, Y, kind, p, out_ptr, ldo, ws_ptr, ws_bytes, flags, stream):
    return load().pcf_cross(ctypes.byref(X), ctypes.byref(Y), kind, p, out_ptr, ldo,
                            ws_ptr, ws_bytes, flags, stream)


def pcf_cross_workspace_bytes(X, Y):
    out = ctypes.c_size_t(0)
    check(load().pcf_cross_workspace_bytes(ctypes.byref(X), ctypes.byref(Y),
                                           ctypes.byref(out)))
    return out.value


def pcf_validate(X, ws_ptr, ws_bytes, stream):
    bad = ctypes.c_int64(-1)
    check(load().pcf_validate(ctypes.byref(X), ctypes.byref(bad), ws_ptr, ws_bytes, stream))
    return bad.value


def pcf_plan_inspect(n, offsets_host_ptr, dtype, window, backward, blocks_cap=0,
                     blocks_buf_ptr=None):
    nb, ns, nt = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    check(load().pcf_plan_inspect(n, offsets_host_ptr, dtype,
                                  ctypes.byref(window) if window else None,
                                  int(backward), ctypes.byref(nb), ctypes.byref(ns),
                                  ctypes.byref(nt), blocks_buf_ptr, blocks_cap))
    return nb.value, ns.value, nt.value
