// single.hip -- per-PCF operations: functionals of one PCF at a time (paper,
// Section 3.2 "PCF integrals": F(f) = r(int_a^b h(f(t)) dt) for every PCF of
// a set), the restriction of a set to an integration range [a, b), and the
// time warp of a set for a time-dependent h = h0(a, b) w(t).
//
// Segment iteration (Algorithm IterateSegments) walks a PCF's pieces and
// adds (r - l) h(v) per segment [l, r) of [a, b). Piece k of a PCF is
// [t_k, t_{k+1}) (t_n = inf), so its segment is that piece clipped to
// [a, b); the segments of all pieces, summed, are the walk's segments. One
// wave per PCF: lane j takes pieces j, j + 64, ..., and the 64 partial sums
// are added by a fixed butterfly, so results do not depend on timing. With
// b = inf the unbounded last piece adds 0 when h(v_last) = 0 and an infinity
// of the sign of h(v_last) otherwise. The work is one pass over the set's
// rows: HBM-bound (16 B per FP64 row, 8 B per FP32 row, plus the offsets).
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace pcf {

// h of the single-PCF kinds: SK_VALUE h(v) = v; SK_ABS |v|; SK_SQR v^2;
// SK_POW |v|^p.
// SK_SUP: sup |v| over the segments (the L_inf norm), not an integral.
enum { SK_VALUE = 0, SK_ABS = 1, SK_SQR = 2, SK_POW = 3, SK_SUP = 4 };

template <int SK>
__device__ __forceinline__ double h_single(double v, double p)
{
    if constexpr (SK == SK_VALUE)
        return v;
    else if constexpr (SK == SK_ABS)
        return fabs(v);
    else if constexpr (SK == SK_SQR)
        return v * v;
    else
        return pow(fabs(v), p);
}

// Sum over the 64 lanes of a wave by a butterfly of fixed shape.
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ double wave_max(double x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double y = __shfl_xor(x, o, 64);
        x = y > x ? y : x;
    }
    return x;
}

// Rows a lane loads per round: lane j takes rows j, j + 64, ..., j + 64 (kRound
// - 1) of the round, all loads issued before any is used, so a PCF of up to
// 64 kRound rows costs one memory round trip instead of one per 64 rows. The
// lane adds its rows in increasing order, as one row at a time would.
constexpr int kRound = 4;

template <typename T, int SK>
__global__ void single_functional(SingleArgs a)
{
    const T *__restrict__ t = reinterpret_cast<const T *>(a.t);
    const T *__restrict__ v = reinterpret_cast<const T *>(a.v);
    T *__restrict__ out = reinterpret_cast<T *>(a.out);
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    // this wave's PCF row range, loaded one PCF ahead
    int64_t o0 = 0, o1 = 0;
    if (i < a.n) {
        o0 = a.offsets[i];
        o1 = a.offsets[i + 1];
    }
    for (; i < a.n; i += nwaves) {
        const int64_t in = i + nwaves;
        int64_t n0 = 0, n1 = 0;
        if (in < a.n) {
            n0 = a.offsets[in];
            n1 = a.offsets[in + 1];
        }
        double acc = 0.0;
        int tail = 0;  // sign of h on an unbounded last piece
        for (int64_t base = o0 + lane; base < o1; base += 64 * kRound) {
            double tk[kRound], tn[kRound], vk[kRound];
#pragma unroll
            for (int u = 0; u < kRound; ++u) {
                const int64_t k = base + 64 * u;
                tk[u] = tn[u] = vk[u] = 0.0;
                if (k < o1) {
                    tk[u] = (double)t[k];
                    tn[u] = k + 1 < o1 ? (double)t[k + 1] : INFINITY;
                    vk[u] = (double)v[k];
                }
            }
#pragma unroll
            for (int u = 0; u < kRound; ++u) {
                if (base + 64 * u >= o1)
                    break;
                const double l = tk[u] > a.a ? tk[u] : a.a;
                const double r = tn[u] < a.b ? tn[u] : a.b;
                if (r > l) {
                    if constexpr (SK == SK_SUP) {
                        const double av = fabs(vk[u]);
                        acc = av > acc ? av : acc;
                    } else {
                        const double hv = h_single<SK>(vk[u], a.p);
                        if (r == INFINITY)
                            tail = hv > 0.0 ? 1 : (hv < 0.0 ? -1 : 0);
                        else
                            acc += (r - l) * hv;
                    }
                }
            }
        }
        if constexpr (SK == SK_SUP)
            acc = wave_max(acc);
        else
            acc = wave_sum(acc);
        // the tail is set on one lane at most (the last piece)
        int tl = tail;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            tl |= __shfl_xor(tl, o, 64);
        if (lane == 0) {
            double res = tl == 0 ? acc : (tl > 0 ? INFINITY : -INFINITY);
            if (a.root == 1)
                res = sqrt(res);
            else if (a.root == 2)
                res = pow(res, 1.0 / a.p);
            out[i] = (T)res;
        }
        o0 = n0;
        o1 = n1;
    }
}

template <typename T, int SK>
static hipError_t launch_single_t(const SingleArgs &a, hipStream_t s)
{
    // one wave a workgroup (measured 4 % faster than four waves)
    int64_t blocks = a.n;
    if (blocks > 32768)
        blocks = 32768;
    hipLaunchKernelGGL((single_functional<T, SK>), dim3((unsigned)blocks), dim3(64), 0,
                       s, a);
    return hipGetLastError();
}

hipError_t launch_single(bool f64, int sk, const SingleArgs &a, hipStream_t s)
{
    if (a.n <= 0)
        return hipSuccess;
    if (f64) {
        switch (sk) {
        case SK_VALUE: return launch_single_t<double, SK_VALUE>(a, s);
        case SK_ABS: return launch_single_t<double, SK_ABS>(a, s);
        case SK_SQR: return launch_single_t<double, SK_SQR>(a, s);
        case SK_SUP: return launch_single_t<double, SK_SUP>(a, s);
        default: return launch_single_t<double, SK_POW>(a, s);
        }
    }
    switch (sk) {
    case SK_VALUE: return launch_single_t<float, SK_VALUE>(a, s);
    case SK_ABS: return launch_single_t<float, SK_ABS>(a, s);
    case SK_SQR: return launch_single_t<float, SK_SQR>(a, s);
    case SK_SUP: return launch_single_t<float, SK_SUP>(a, s);
    default: return launch_single_t<float, SK_POW>(a, s);
    }
}

// ---------------------------------------------------------------------------
// Restriction to an integration range (paper, Section 2.2: combination
// integrals over [a, b)): f 1_[a,b) is again a PCF, and since h(0, 0) = 0
// for every kind, int_a^b h(f, g) = int_0^inf h(f 1_[a,b), g 1_[a,b)). Its
// rows: (0, 0) and (a, f(a)) when a > 0, else (0, f(0)); the rows of f with
// a < t_k < b; (b, 0) when b is finite. a and b are taken in the set's
// precision.

// Rows of f before and at x: the number of times t_k <= x (strict: t_k < x).
template <typename T>
__device__ __forceinline__ int64_t count_le(const T *t, int64_t n, T x, bool strict)
{
    int64_t lo = 0, hi = n;  // the answer lies in [lo, hi]
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const bool in = strict ? (t[mid] < x) : (t[mid] <= x);
        if (in)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Row range [k_a + 1, k_b) of the rows kept from f, and k_a (the piece
// holding a).
template <typename T>
__device__ __forceinline__ void kept_rows(const T *t, int64_t n, T a, T b, bool b_finite,
                                          int64_t &ka, int64_t &kb)
{
    ka = count_le(t, n, a, false) - 1;  // t_0 = 0 <= a
    kb = b_finite ? count_le(t, n, b, true) : n;
}

template <typename T>
__global__ void restrict_count(const int64_t *__restrict__ offsets, int64_t n,
                               const T *__restrict__ t, double a, double b,
                               int64_t *__restrict__ counts)
{
    const T ta = (T)a, tb = (T)b;
    const bool bf = !(b == INFINITY);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = offsets[i], ni = offsets[i + 1] - o;
        int64_t ka, kb;
        kept_rows(t + o, ni, ta, tb, bf, ka, kb);
        const int64_t mid = kb - (ka + 1) > 0 ? kb - (ka + 1) : 0;
        counts[i + 1] = (ta > T(0) ? 2 : 1) + mid + (bf ? 1 : 0);
        if (i == 0)
            counts[0] = 0;
    }
}

// One wave per PCF: lane 0 writes the head and tail rows, the lanes copy the
// kept rows.
template <typename T>
__global__ void restrict_fill(const int64_t *__restrict__ offsets, int64_t n,
                              const T *__restrict__ t, const T *__restrict__ v,
                              double a, double b, const int64_t *__restrict__ out_off,
                              T *__restrict__ t_out, T *__restrict__ v_out)
{
    const T ta = (T)a, tb = (T)b;
    const bool bf = !(b == INFINITY);
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n;
         i += nwaves) {
        const int64_t o = offsets[i], ni = offsets[i + 1] - o;
        int64_t ka, kb;
        kept_rows(t + o, ni, ta, tb, bf, ka, kb);
        int64_t w = out_off[i];
        const int head = ta > T(0) ? 2 : 1;
        if (lane == 0) {
            if (head == 2) {
                t_out[w] = T(0);
                v_out[w] = T(0);
                t_out[w + 1] = ta;
                v_out[w + 1] = v[o + ka];
            } else {
                t_out[w] = T(0);
                v_out[w] = v[o];
            }
        }
        w += head;
        for (int64_t k = ka + 1 + lane; k < kb; k += 64) {
            t_out[w + (k - ka - 1)] = t[o + k];
            v_out[w + (k - ka - 1)] = v[o + k];
        }
        if (lane == 0 && bf) {
            const int64_t last = out_off[i + 1] - 1;
            t_out[last] = tb;
            v_out[last] = T(0);
        }
    }
}

// Gradients through a restriction. Y = X 1_[a,b) holds, per PCF, a head row
// (a, v_ka) (after (0, 0) when a > 0; (0, v_0) when a = 0), X's rows
// ka+1 .. kb-1, and (b, 0) when b is finite. Given dL/dt, dL/dv of Y's rows
// (FP64), X's rows get: a kept row, its own; row ka, the head row's value
// gradient; every other row 0 (the times 0, a, b and the added values are
// constants, and rows outside the range do not reach Y). The last value is a
// fixed parameter, as in the adjoint. One wave per PCF.
template <typename T>
__global__ void restrict_backward(const int64_t *__restrict__ offsets, int64_t n,
                                  const T *__restrict__ t, double a, double b,
                                  const int64_t *__restrict__ y_off,
                                  const double *__restrict__ gt_y,
                                  const double *__restrict__ gv_y, double *__restrict__ gt_x,
                                  double *__restrict__ gv_x)
{
    const T ta = (T)a, tb = (T)b;
    const bool bf = !(b == INFINITY);
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n;
         i += nwaves) {
        const int64_t o = offsets[i], ni = offsets[i + 1] - o;
        int64_t ka, kb;
        kept_rows(t + o, ni, ta, tb, bf, ka, kb);
        const int head = ta > T(0) ? 2 : 1;
        const int64_t w = y_off[i] + head;  // Y's row of X's row ka + 1
        for (int64_t k = lane; k < ni; k += 64) {
            double gt = 0.0, gv = 0.0;
            if (k > ka && k < kb) {
                gt = gt_y[w + (k - ka - 1)];
                gv = gv_y[w + (k - ka - 1)];
            }
            if (k == ka)
                gv = gv_y[w - 1];  // the head row (a, v_ka)
            if (k == ni - 1)
                gv = 0.0;  // the last value is fixed (0 by the data contract)
            gt_x[o + k] = gt;
            gv_x[o + k] = gv;
        }
    }
}

hipError_t launch_restrict_count(bool f64, const int64_t *offsets, int64_t n,
                                 const void *t, double a, double b, int64_t *counts,
                                 hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    if (f64)
        hipLaunchKernelGGL(restrict_count<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const double *)t, a, b, counts);
    else
        hipLaunchKernelGGL(restrict_count<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const float *)t, a, b, counts);
    return hipGetLastError();
}

hipError_t launch_restrict_backward(bool f64, const int64_t *offsets, int64_t n,
                                    const void *t, double a, double b, const int64_t *y_off,
                                    const double *gt_y, const double *gv_y, double *gt_x,
                                    double *gv_x, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t blocks = (n + 3) / 4;
    if (blocks > 8192)
        blocks = 8192;
    if (f64)
        hipLaunchKernelGGL(restrict_backward<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const double *)t, a, b, y_off, gt_y, gv_y, gt_x, gv_x);
    else
        hipLaunchKernelGGL(restrict_backward<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const float *)t, a, b, y_off, gt_y, gv_y, gt_x, gv_x);
    return hipGetLastError();
}

hipError_t launch_restrict_fill(bool f64, const int64_t *offsets, int64_t n,
                                const void *t, const void *v, double a, double b,
                                const int64_t *out_off, void *t_out, void *v_out,
                                hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t blocks = (n + 3) / 4;
    if (blocks > 8192)
        blocks = 8192;
    if (f64)
        hipLaunchKernelGGL(restrict_fill<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const double *)t, (const double *)v, a, b,
                           out_off, (double *)t_out, (double *)v_out);
    else
        hipLaunchKernelGGL(restrict_fill<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const float *)t, (const float *)v, a, b,
                           out_off, (float *)t_out, (float *)v_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Time warp (Section 3, time-dependent h with an antiderivative H in t;
// Section 2.2, weighted L_p and inner products). For h = h0(a, b) w(t),
// H = h0 W with W(t) = int_0^t w, and a cell [l, r) of the merge adds
// h0 (W(r) - W(l)). Carrying every breakpoint t_k to tau_k = W(t_k) turns
// that into h0 (tau_r - tau_l), the contribution of the plain merge on the
// warped set: W is evaluated once per breakpoint instead of twice per cell
// and pair, and the pairwise kernels run unchanged. Weights:
//   WK_EXP  w(t) = exp(-c t), c > 0:  W(t) = -expm1(-c t) / c
//   WK_POW  w(t) = t^c, c > -1:       W(t) = t^(c+1) / (c+1)
// W is increasing, but rounded values can tie: a run of rows with one tau
// keeps only its last row (its value holds on the next piece of positive
// width), so the warped set is strictly increasing again. A tau that is not
// finite, or decreases, marks the PCF bad (count -1).
enum { WK_EXP = 1, WK_POW = 2 };

template <typename T>
__device__ __forceinline__ T warped(const T *t, int64_t k, int wk, double c)
{
    if (k == 0)
        return T(0);
    const double x = (double)t[k];
    const double w = wk == WK_EXP ? -expm1(-c * x) / c : pow(x, c + 1.0) / (c + 1.0);
    return (T)w;
}

// One 64-row chunk of a PCF's warped rows: tau of row base + lane, whether
// that row is kept, and whether it breaks monotonicity or finiteness.
template <typename T>
__device__ __forceinline__ void warp_chunk(const T *t, int64_t ni, int64_t base, int lane,
                                           int wk, double c, T &tau, bool &keep, bool &bad)
{
    const int64_t k = base + lane;
    tau = k < ni ? warped(t, k, wk, c) : T(0);
    T nxt = __shfl_down(tau, 1, 64);
    if (lane == 63 && k + 1 < ni)
        nxt = warped(t, k + 1, wk, c);
    const bool in = k < ni, last = k + 1 == ni;
    keep = in && (last || nxt > tau);
    bad = in && (!isfinite(tau) || (!last && nxt < tau));
}

template <typename T>
__global__ void warp_count(const int64_t *__restrict__ offsets, int64_t n,
                           const T *__restrict__ t, int wk, double c,
                           int64_t *__restrict__ counts)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n;
         i += nwaves) {
        const int64_t o = offsets[i], ni = offsets[i + 1] - o;
        int64_t kept = 0;
        bool anybad = false;
        for (int64_t base = 0; base < ni; base += 64) {
            T tau;
            bool keep, bad;
            warp_chunk(t + o, ni, base, lane, wk, c, tau, keep, bad);
            kept += __popcll(__ballot(keep));
            anybad = anybad || __ballot(bad) != 0;
        }
        if (lane == 0) {
            counts[i + 1] = anybad ? -1 : kept;
            if (i == 0)
                counts[0] = 0;
        }
    }
}

// Gradients through a time warp: Y's kept rows are (W(t_k), v_k), so X's
// row k gets dL/dt = dL/dtau w(t_k) (W' = w; t_0 = 0 is fixed) and dL/dv as
// given; a row dropped because its rounded tau ties the next one's (a piece
// of zero width in Y) gets 0. One wave per PCF, the rows decided as in
// warp_fill.
template <typename T>
__global__ void warp_backward(const int64_t *__restrict__ offsets, int64_t n,
                              const T *__restrict__ t, int wk, double c,
                              const int64_t *__restrict__ y_off,
                              const double *__restrict__ gt_y,
                              const double *__restrict__ gv_y, double *__restrict__ gt_x,
                              double *__restrict__ gv_x)
{
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n;
         i += nwaves) {
        const int64_t o = offsets[i], ni = offsets[i + 1] - o;
        int64_t w = y_off[i];
        const int64_t end = y_off[i + 1];
        for (int64_t base = 0; base < ni; base += 64) {
            T tau;
            bool keep, bad;
            warp_chunk(t + o, ni, base, lane, wk, c, tau, keep, bad);
            const uint64_t m = __ballot(keep);
            const int64_t pos = w + __popcll(m & below);
            const int64_t k = base + lane;
            if (k < ni) {
                double gt = 0.0, gv = 0.0;
                if (keep && pos < end) {
                    gv = gv_y[pos];
                    if (k > 0) {
                        const double x = (double)t[o + k];
                        gt = gt_y[pos] * (wk == WK_EXP ? exp(-c * x) : pow(x, c));
                    }
                }
                gt_x[o + k] = gt;
                gv_x[o + k] = gv;
            }
            w += __popcll(m);
        }
    }
}

template <typename T>
__global__ void warp_fill(const int64_t *__restrict__ offsets, int64_t n,
                          const T *__restrict__ t, const T *__restrict__ v, int wk,
                          double c, const int64_t *__restrict__ out_off,
                          T *__restrict__ t_out, T *__restrict__ v_out)
{
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n;
         i += nwaves) {
        const int64_t o = offsets[i], ni = offsets[i + 1] - o;
        int64_t w = out_off[i];
        const int64_t end = out_off[i + 1];  // the count pass made the same decisions
        for (int64_t base = 0; base < ni; base += 64) {
            T tau;
            bool keep, bad;
            warp_chunk(t + o, ni, base, lane, wk, c, tau, keep, bad);
            const uint64_t m = __ballot(keep);
            const int64_t pos = w + __popcll(m & below);
            if (keep && pos < end) {
                t_out[pos] = tau;
                v_out[pos] = v[o + base + lane];
            }
            w += __popcll(m);
        }
    }
}

hipError_t launch_warp_count(bool f64, const int64_t *offsets, int64_t n, const void *t,
                             int wk, double c, int64_t *counts, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t blocks = (n + 3) / 4;
    if (blocks > 8192)
        blocks = 8192;
    if (f64)
        hipLaunchKernelGGL(warp_count<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const double *)t, wk, c, counts);
    else
        hipLaunchKernelGGL(warp_count<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const float *)t, wk, c, counts);
    return hipGetLastError();
}

hipError_t launch_warp_fill(bool f64, const int64_t *offsets, int64_t n, const void *t,
                            const void *v, int wk, double c, const int64_t *out_off,
                            void *t_out, void *v_out, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t blocks = (n + 3) / 4;
    if (blocks > 8192)
        blocks = 8192;
    if (f64)
        hipLaunchKernelGGL(warp_fill<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const double *)t, (const double *)v, wk, c,
                           out_off, (double *)t_out, (double *)v_out);
    else
        hipLaunchKernelGGL(warp_fill<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const float *)t, (const float *)v, wk, c,
                           out_off, (float *)t_out, (float *)v_out);
    return hipGetLastError();
}


hipError_t launch_warp_backward(bool f64, const int64_t *offsets, int64_t n, const void *t,
                                int wk, double c, const int64_t *y_off, const double *gt_y,
                                const double *gv_y, double *gt_x, double *gv_x, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t blocks = (n + 3) / 4;
    if (blocks > 8192)
        blocks = 8192;
    if (f64)
        hipLaunchKernelGGL(warp_backward<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const double *)t, wk, c, y_off, gt_y, gv_y, gt_x, gv_x);
    else
        hipLaunchKernelGGL(warp_backward<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           offsets, n, (const float *)t, wk, c, y_off, gt_y, gv_y, gt_x, gv_x);
    return hipGetLastError();
}


// The root of a sum of terms (pcf_pairwise_terms): x -> x^(1/q) (sqrt for
// q = 2) over a region of the output, one thread per entry.
template <typename T>
__global__ void apply_root(T *__restrict__ out, int64_t rows, int64_t cols, int64_t ldo,
                          double q, int upper, int64_t i0, int64_t j0)
{
    const int64_t total = rows * cols;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = k / cols, c = k - r * cols;
        if (upper && i0 + r > j0 + c)
            continue;
        T *x = out + r * ldo + c;
        *x = q == 2.0 ? (T)sqrt((double)*x) : (T)pow((double)*x, 1.0 / q);
    }
}

hipError_t launch_apply_root(bool f64, void *out, int64_t rows, int64_t cols, int64_t ldo,
                             double q, bool upper, int64_t i0, int64_t j0, hipStream_t s)
{
    if (rows <= 0 || cols <= 0)
        return hipSuccess;
    int64_t blocks = (rows * cols + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    if (f64)
        hipLaunchKernelGGL(apply_root<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (double *)out, rows, cols, ldo, q, upper ? 1 : 0, i0, j0);
    else
        hipLaunchKernelGGL(apply_root<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (float *)out, rows, cols, ldo, q, upper ? 1 : 0, i0, j0);
    return hipGetLastError();
}
}  // namespace pcf
