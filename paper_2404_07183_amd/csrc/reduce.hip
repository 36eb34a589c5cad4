// reduce.hip -- reductions of groups of PCFs (paper, Section 2.1
// "Combinations and reductions"; Section 4, reduction trees and Algorithm
// ReducePair): sum, max and min by the induced reduction, mean = sum / n and
// the sample standard deviation sqrt(sum_i (f_i - mean)^2 / (n - 1)).
//
// Tree. A group of M PCFs is reduced by a binary tree: at level l the items
// 2j and 2j+1 (each covering 2^l consecutive PCFs) are merged into item j of
// level l+1, and an unpaired last item moves up unchanged. Every group takes
// the same ceil(log2 M_max) levels, one launch per level for all groups.
// Item j of a level writes where its first PCF's rows start: the union of
// two PCFs' breakpoints has at most their total row count, so item ranges
// never overlap and no per-level scan is needed.
//
// Merge. One wave per pair. The merged sequence of the two breakpoint
// lists (ties: the first list first) is cut into 64 x kMergeK positions per
// window; each lane finds its start by a merge-path search and walks
// kMergeK positions. A position opens a cell (a rectangle of ReducePair)
// when the next breakpoint of either list is later; the cell's value is
// h(f(x), g(x)). Lanes write their cells in order after a wave scan of the
// counts. No cell is dropped inside the tree: ReducePair's rule (keep a row
// when t = 0 or its value differs from the previous one) is applied once,
// to the root. That gives the same function and the same minimal rows,
// since the values at each breakpoint do not depend on which rows the
// intermediate PCFs kept.
//
// Standard deviation. For every breakpoint x of the group's root,
// (f_i(x) - mean(x))^2 is summed over i in the tree's order (a binary
// counter over i reproduces the level-by-level pairing), then the root rule
// and x -> sqrt(x / (n - 1)) are applied.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace pcf {

namespace {

constexpr int kMergeK = 4;

template <typename T, int OP>
__device__ __forceinline__ T red_op(T a, T b)
{
    if constexpr (OP == RO_MAX)
        return a >= b ? a : b;
    else if constexpr (OP == RO_MIN)
        return a <= b ? a : b;
    else
        return a + b;
}

// Group b holding wave item w: the last b with prefix[b] <= w.
__device__ __forceinline__ int32_t group_of(const int64_t *prefix, int32_t B, int64_t w)
{
    int32_t lo = 0, hi = B - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int wave_excl_scan(int c, int lane, int &total)
{
    int incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o)
            incl += y;
    }
    total = __shfl(incl, 63, 64);
    return incl - c;
}

}  // namespace

__global__ void red_init_counts(const int64_t *__restrict__ offsets, int64_t n,
                                int64_t *__restrict__ cnt)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        cnt[i] = offsets[i + 1] - offsets[i];
}

template <typename T, int OP>
__global__ void red_level(RedLevelArgs a)
{
    const T *__restrict__ tin = reinterpret_cast<const T *>(a.tin);
    const T *__restrict__ vin = reinterpret_cast<const T *>(a.vin);
    T *__restrict__ tout = reinterpret_cast<T *>(a.tout);
    T *__restrict__ vout = reinterpret_cast<T *>(a.vout);
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nitems = a.items[a.B];
    const int64_t span = (int64_t)1 << a.level;
    const T inf = (T)INFINITY;
    for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < nitems;
         w += nwaves) {
        const int32_t b = group_of(a.items, a.B, w);
        const int64_t j = w - a.items[b];
        const int64_t ge = a.groups[b + 1];
        const int64_t iA = a.groups[b] + 2 * j * span, iB = iA + span;
        const int64_t sA = a.offsets[iA], nA = a.cnt[iA];
        if (iB >= ge) {  // unpaired: moves up unchanged
            for (int64_t k = lane; k < nA; k += 64) {
                tout[sA + k] = tin[sA + k];
                vout[sA + k] = vin[sA + k];
            }
            continue;
        }
        const int64_t sB = a.offsets[iB], nB = a.cnt[iB];
        const T *tA = tin + sA, *vA = vin + sA, *tB = tin + sB, *vB = vin + sB;
        const int64_t total = nA + nB;
        int64_t out = 0;
        for (int64_t wb = 0; wb < total; wb += 64 * kMergeK) {
            const int64_t d = wb + (int64_t)lane * kMergeK;
            T xs[kMergeK], vs[kMergeK];
            unsigned starts = 0;
            if (d < total) {
                int64_t lo = d - nB > 0 ? d - nB : 0, hi = d < nA ? d : nA;
                while (lo < hi) {  // A's share of the first d merged positions
                    const int64_t mid = (lo + hi) >> 1;
                    if (tA[mid] <= tB[d - 1 - mid])
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                int64_t i = lo, jj = d - lo;
#pragma unroll
                for (int q = 0; q < kMergeK; ++q) {
                    if (d + q < total) {
                        T x;
                        if (i < nA && (jj >= nB || tA[i] <= tB[jj]))
                            x = tA[i++];
                        else
                            x = tB[jj++];
                        const T ta = i < nA ? tA[i] : inf, tb = jj < nB ? tB[jj] : inf;
                        if (x < (ta < tb ? ta : tb)) {
                            starts |= 1u << q;
                            xs[q] = x;
                            vs[q] = red_op<T, OP>(vA[i > 0 ? i - 1 : 0], vB[jj > 0 ? jj - 1 : 0]);
                        }
                    }
                }
            }
            int wtotal;
            int64_t pos = out + wave_excl_scan(__popc(starts), lane, wtotal);
#pragma unroll
            for (int q = 0; q < kMergeK; ++q) {
                if (starts & (1u << q)) {
                    tout[sA + pos] = xs[q];
                    vout[sA + pos] = vs[q];
                    ++pos;
                }
            }
            out += wtotal;
        }
        if (lane == 0)
            a.cnt[iA] = out;
    }
}

// Sum over i of (f_i(x) - mean(x))^2 at every root breakpoint x, in the
// tree's order.
template <typename T>
__global__ void red_std_terms(RedStdArgs a)
{
#pragma clang fp contract(off)
    const T *__restrict__ t = reinterpret_cast<const T *>(a.t);
    const T *__restrict__ v = reinterpret_cast<const T *>(a.v);
    const T *__restrict__ rt = reinterpret_cast<const T *>(a.rt);
    const T *__restrict__ rv = reinterpret_cast<const T *>(a.rv);
    T *__restrict__ q = reinterpret_cast<T *>(a.q);
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.rows;
         r += (int64_t)gridDim.x * blockDim.x) {
        // the group whose root holds row r: last b with offsets[groups[b]] <= r
        int32_t lo = 0, hi = a.B - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (a.offsets[a.groups[mid]] <= r)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int64_t gb = a.groups[lo], ge = a.groups[lo + 1];
        const int64_t u = r - a.offsets[gb];
        if (u >= a.cnt[gb])
            continue;
        const T x = rt[r];
        const T mean = rv[r] / (T)(ge - gb);
        T st[64];
        int ht[64];
        int top = 0;
        for (int64_t i = gb; i < ge; ++i) {
            const int64_t o = a.offsets[i], ni = a.offsets[i + 1] - o;
            int64_t l = 0, h = ni;  // rows with t <= x
            while (l < h) {
                const int64_t m = (l + h) >> 1;
                if (t[o + m] <= x)
                    l = m + 1;
                else
                    h = m;
            }
            const T d = v[o + (l > 0 ? l - 1 : 0)] - mean;
            T s = d * d;
            int hs = 0;
            while (top > 0 && ht[top - 1] == hs) {
                s = st[top - 1] + s;
                --top;
                ++hs;
            }
            st[top] = s;
            ht[top] = hs;
            ++top;
        }
        T acc = st[top - 1];
        for (int k = top - 2; k >= 0; --k)
            acc = st[k] + acc;
        q[r] = acc;
    }
}

// Root rows kept by ReducePair's rule (all rows of a one-PCF group), and
// their values after the group's transformation.
template <typename T>
__device__ __forceinline__ T red_finish(int op, T x, int64_t m)
{
    if (op == RO_MEAN)
        return x / (T)m;
    if (op == RO_STD)
        return sqrt(x / (T)(m - 1));
    return x;
}

template <typename T>
__global__ void red_emit(RedEmitArgs a)
{
    const T *__restrict__ rt = reinterpret_cast<const T *>(a.rt);
    const T *__restrict__ rv = reinterpret_cast<const T *>(a.rv);
    T *__restrict__ t_out = reinterpret_cast<T *>(a.t_out);
    T *__restrict__ v_out = reinterpret_cast<T *>(a.v_out);
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; b < a.B;
         b += nwaves) {
        const int64_t gb = a.groups[b], m = a.groups[b + 1] - gb;
        const int64_t s = a.offsets[gb], c = a.cnt[gb];
        int64_t w = a.fill ? a.out_off[b] : 0;
        const int64_t end = a.fill ? a.out_off[b + 1] : 0;
        for (int64_t base = 0; base < c; base += 64) {
            const int64_t k = base + lane;
            const bool keep = k < c && (m == 1 || k == 0 || rv[s + k] != rv[s + k - 1]);
            const uint64_t mask = __ballot(keep);
            if (a.fill) {
                const int64_t pos = w + __popcll(mask & below);
                if (keep && pos < end) {
                    t_out[pos] = rt[s + k];
                    v_out[pos] = red_finish<T>(a.op, rv[s + k], m);
                }
            }
            w += __popcll(mask);
        }
        if (!a.fill && lane == 0) {
            a.counts[b + 1] = w;
            if (b == 0)
                a.counts[0] = 0;
        }
    }
}

static int64_t grid_for(int64_t units, int64_t per_block, int64_t cap)
{
    int64_t g = (units + per_block - 1) / per_block;
    return g < 1 ? 1 : (g > cap ? cap : g);
}

hipError_t launch_red_init(const int64_t *offsets, int64_t n, int64_t *cnt, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(red_init_counts, dim3((unsigned)grid_for(n, 256, 4096)), dim3(256), 0,
                       s, offsets, n, cnt);
    return hipGetLastError();
}

hipError_t launch_red_level(bool f64, int op, const RedLevelArgs &a, int64_t nitems,
                            hipStream_t s)
{
    if (nitems <= 0)
        return hipSuccess;
    const dim3 g((unsigned)grid_for(nitems, 4, 16384)), blk(256);
    const int o = op == RO_MAX ? RO_MAX : (op == RO_MIN ? RO_MIN : RO_SUM);
    if (f64) {
        if (o == RO_MAX)
            hipLaunchKernelGGL((red_level<double, RO_MAX>), g, blk, 0, s, a);
        else if (o == RO_MIN)
            hipLaunchKernelGGL((red_level<double, RO_MIN>), g, blk, 0, s, a);
        else
            hipLaunchKernelGGL((red_level<double, RO_SUM>), g, blk, 0, s, a);
    } else {
        if (o == RO_MAX)
            hipLaunchKernelGGL((red_level<float, RO_MAX>), g, blk, 0, s, a);
        else if (o == RO_MIN)
            hipLaunchKernelGGL((red_level<float, RO_MIN>), g, blk, 0, s, a);
        else
            hipLaunchKernelGGL((red_level<float, RO_SUM>), g, blk, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_red_std(bool f64, const RedStdArgs &a, hipStream_t s)
{
    if (a.rows <= 0)
        return hipSuccess;
    const dim3 g((unsigned)grid_for(a.rows, 256, 8192)), blk(256);
    if (f64)
        hipLaunchKernelGGL(red_std_terms<double>, g, blk, 0, s, a);
    else
        hipLaunchKernelGGL(red_std_terms<float>, g, blk, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_red_emit(bool f64, const RedEmitArgs &a, hipStream_t s)
{
    if (a.B <= 0)
        return hipSuccess;
    const dim3 g((unsigned)grid_for(a.B, 4, 8192)), blk(256);
    if (f64)
        hipLaunchKernelGGL(red_emit<double>, g, blk, 0, s, a);
    else
        hipLaunchKernelGGL(red_emit<float>, g, blk, 0, s, a);
    return hipGetLastError();
}

}  // namespace pcf
