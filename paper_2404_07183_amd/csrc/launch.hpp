// launch.hpp -- kernel argument blocks and launcher entry points shared by
// the C-ABI layer (abi.hip) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace pcf {

// h codes of the combination integral (Section 2.2 of the paper).
// kPowInt: |a-b|^p for an integer p, by squaring; kPowHalf: p = k + 1/2, by
// squaring and one square root; kPow: any other p, as 2^(p log2 |a-b|) (FP64:
// the series of pow64.hpp; FP32: the hardware base-2 log and exp).
enum HKind : int { kAbs = 0, kSqr = 1, kProd = 2, kPow = 3, kPowHalf = 4, kPowInt = 5 };
// r codes of the combination integral.
enum Root : int { kRootNone = 0, kRootSqrt = 1, kRootPow = 2 };

struct FwdArgs {
    const int64_t *offsets;  // device CSR offsets
    unsigned char *ws;       // workspace (plan + packed records)
    void *out;               // output matrix (dtype of the input)
    double p;                // exponent for kPow
    double inv_p;            // for kRootPow
    int root;                // Root
    int gram;                // 1: diagonal pairs carry work (Gram)
    int accumulate = 0;      // 1: out += coef * value, 2: out = coef * value
    double coef = 1.0;       // (the terms of a sum; no root)
};

struct BwdArgs {
    const int64_t *offsets;
    unsigned char *ws;
    const double *grad_out;  // dL/dF, n x n, leading dimension ldg
    int64_t ldg;
    const double *fwd_out;   // forward result (for the root's chain factor)
    int64_t ldf;
    void *grad_t;            // dL/dt, CSR layout, the set's dtype (accumulated)
    void *grad_v;            // dL/dv, CSR layout, the set's dtype (accumulated)
    double p;
    int chain;               // 1: scale by dF/dI = (1/p) I^(1/p - 1)
    int gram;                // 1: diagonal pairs carry work (Gram)
    int64_t n;               // PCFs in the set
    int fixed;               // 1: deterministic: 64-bit fixed-point sums at
                             // the set's scales (FP64: in grad_t, grad_v; FP32:
                             // in the workspace, off_acc) until
                             // launch_adj_finish (needs launch_adj_bounds first)
};

template <typename T>
hipError_t launch_pack(const int64_t *offsets, int64_t n, const void *t,
                       const void *v, unsigned char *ws, int64_t P,
                       hipStream_t s, int64_t rec_base = 0);
hipError_t launch_concat_offsets(const int64_t *xo, int64_t nx, const int64_t *yo,
                                 int64_t ny, int64_t *out, hipStream_t s);
template <typename T>
hipError_t launch_validate(const int64_t *offsets, int64_t n, const void *t,
                           const void *v, unsigned char *ws, int64_t P,
                           hipStream_t s);
// Single-PCF functionals (single.hip).
struct SingleArgs {
    const int64_t *offsets;
    int64_t n;
    const void *t, *v;
    void *out;
    double a, b;  // integration bounds, 0 <= a < b <= inf
    double p;
    int root;     // 0: none, 1: sqrt, 2: x^(1/p)
};
hipError_t launch_single(bool f64, int sk, const SingleArgs &a, hipStream_t s);
hipError_t launch_restrict_count(bool f64, const int64_t *offsets, int64_t n,
                                 const void *t, double a, double b, int64_t *counts,
                                 hipStream_t s);
hipError_t launch_restrict_fill(bool f64, const int64_t *offsets, int64_t n,
                                const void *t, const void *v, double a, double b,
                                const int64_t *out_off, void *t_out, void *v_out,
                                hipStream_t s);
hipError_t launch_warp_count(bool f64, const int64_t *offsets, int64_t n, const void *t,
                             int wk, double c, int64_t *counts, hipStream_t s);
hipError_t launch_warp_fill(bool f64, const int64_t *offsets, int64_t n, const void *t,
                            const void *v, int wk, double c, const int64_t *out_off,
                            void *t_out, void *v_out, hipStream_t s);
// gradients through a restriction / a warp: dL/dt, dL/dv (FP64) of the
// transformed set Y (offsets y_off) to those of X's rows
hipError_t launch_restrict_backward(bool f64, const int64_t *offsets, int64_t n,
                                    const void *t, double a, double b, const int64_t *y_off,
                                    const double *gt_y, const double *gv_y, double *gt_x,
                                    double *gv_x, hipStream_t s);
hipError_t launch_warp_backward(bool f64, const int64_t *offsets, int64_t n, const void *t,
                                int wk, double c, const int64_t *y_off, const double *gt_y,
                                const double *gv_y, double *gt_x, double *gv_x, hipStream_t s);
// x -> x^(1/q) over a rows x cols region of out (leading dimension ldo); with
// upper, only the entries whose global row i0 + r is at most their global
// column j0 + c
hipError_t launch_apply_root(bool f64, void *out, int64_t rows, int64_t cols, int64_t ldo,
                             double q, bool upper, int64_t i0, int64_t j0, hipStream_t s);
hipError_t launch_reset(unsigned char *ws, hipStream_t s);
hipError_t launch_forward(bool f64, int hk, const FwdArgs &a, int grid,
                          hipStream_t s);
hipError_t launch_backward(int hk, bool f64, const BwdArgs &a, int grid, hipStream_t s);
// Deterministic adjoint: the set's largest pair weight, |v| and piece length
// into the workspace header (before launch_backward with a.fixed), and the
// fixed-point sums converted to FP64 in place (after it).
hipError_t launch_adj_bounds(bool f64, const BwdArgs &a, hipStream_t s);
hipError_t launch_adj_finish(int hk, bool f64, const BwdArgs &a, int64_t P, hipStream_t s);
// Clears an FP32 plan's deterministic sums (2 P words in the workspace).
hipError_t launch_adj_acc(const BwdArgs &a, int64_t P, hipStream_t s);
hipError_t launch_zero(double *p, int64_t n, hipStream_t s);
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s);
// Raises a kernel's dynamic-LDS limit to `bytes` once per device (thread
// safe: concurrent first calls from several host threads all wait for it).
hipError_t ensure_dynamic_lds(const void *kernel, int bytes);
size_t tile_shared_bytes(int rec_bytes, bool backward);

}  // namespace pcf
