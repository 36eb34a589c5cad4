// reduce.hip -- reductions of groups of PCFs (paper, Section 2.1
// "Combinations and reductions"; Section 4, reduction trees and Algorithm
// ReducePair): sum, max and min by the induced reduction, mean = sum / n and
// the sample standard deviation sqrt(sum_i (f_i - mean)^2 / (n - 1)); and
// the combinations h_*(x_i, y_i) of two sets (also a - b, ab, (a - b)^2) as
// reductions of the interleaved set in groups of two.
//
// Tree. A group of M PCFs is reduced by a binary tree: at level l the items
// 2j and 2j+1 (each covering 2^l consecutive PCFs) are merged into item j of
// level l+1, and an unpaired last item moves up unchanged. Every group takes
// the same ceil(log2 M_max) levels, one launch per level for all groups.
//
// Merge without compaction. A level keeps every position of the merged
// breakpoint lists (ties: the first list first), so item j of level l+1
// holds exactly the rows of its 2^(l+1) PCFs, in the same place: position q
// of a pair is row offsets[first PCF] + q of the output buffer. Every row
// with time x carries h(f(x), g(x)): a list's value at x is its next row's
// when that row also lies at x (all rows at one time carry the same value,
// by induction from the strictly increasing inputs), else its last row's.
// Positions are independent given the merge state, so one launch per level
// covers all rows of all pairs: a lane walks kMergeK consecutive rows after
// a merge-path search, moving on to the next pair in place when it crosses
// one. ReducePair's row rule (keep t = 0 and value changes) is applied once,
// to the root, where runs of rows at one time collapse to their first: the
// same function and the same minimal rows as pruning at every level, since
// the values at each breakpoint do not depend on which rows the
// intermediate PCFs kept. The root pass is cut into chunks of rows; the
// host turns the chunk counts into output offsets.
//
// Standard deviation. For every breakpoint x of the group's root,
// (f_i(x) - mean(x))^2 is summed over i in the tree's order (a binary
// counter over i reproduces the level-by-level pairing), then the root rule
// and x -> sqrt(x / (n - 1)) are applied.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "reduce.hpp"

namespace pcf {

namespace {

// merged positions per lane (4 measured fastest against 2, 8 and 16)
constexpr int kMergeK = 4;
constexpr int kChunkRows = 1024;  // rows per wave in the root pass

template <typename T, int OP>
__device__ __forceinline__ T red_op(T a, T b)
{
    if constexpr (OP == RO_MAX)
        return a >= b ? a : b;
    else if constexpr (OP == RO_MIN)
        return a <= b ? a : b;
    else if constexpr (OP == RO_SUB)
        return a - b;
    else if constexpr (OP == RO_MUL)
        return a * b;
    else if constexpr (OP == RO_SQDIFF)
        return (a - b) * (a - b);
    else
        return a + b;
}

// Last index k in [0, n) with x[k] <= r (x[0] <= r).
__device__ __forceinline__ int64_t last_le(const int64_t *x, int64_t n, int64_t r)
{
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (x[mid] <= r)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The pair of a level that holds a row: its lists' row ranges and the row
// where the pair's output begins.
struct PairAt {
    int64_t b;         // group
    int64_t iA, iE;    // first PCF of the pair, one past its last PCF
    int64_t sA, nA, sB, nB;
};

__device__ __forceinline__ void pair_from(const RedLevelArgs &a, int64_t b, int64_t iA,
                                          int64_t span, PairAt &p)
{
    const int64_t ge = a.groups[b + 1];
    const int64_t iB = iA + span < ge ? iA + span : ge;
    const int64_t iE = iA + 2 * span < ge ? iA + 2 * span : ge;
    p.b = b;
    p.iA = iA;
    p.iE = iE;
    p.sA = a.offsets[iA];
    p.sB = a.offsets[iB];
    p.nA = p.sB - p.sA;
    p.nB = a.offsets[iE] - p.sB;
}

}  // namespace

// Wave-private ordering of LDS accesses (the staging buffers are per wave).
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wave takes 64 * kMergeK consecutive rows; lane l walks rows
// l * kMergeK .. of them. The results go through a wave-private LDS buffer
// so that the stores to memory are coalesced.
template <typename T, int OP>
__global__ __launch_bounds__(256) void red_level(RedLevelArgs a)
{
    const T *__restrict__ tin = reinterpret_cast<const T *>(a.tin);
    const T *__restrict__ vin = reinterpret_cast<const T *>(a.vin);
    T *__restrict__ tout = reinterpret_cast<T *>(a.tout);
    T *__restrict__ vout = reinterpret_cast<T *>(a.vout);
    constexpr int64_t kPerWave = 64 * kMergeK;
    __shared__ T st_t[4][kPerWave], st_v[4][kPerWave];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t span = (int64_t)1 << a.level;
    const int64_t r0g = a.offsets[a.groups[0]], r1g = a.offsets[a.groups[a.B]];
    for (int64_t wb = r0g + ((int64_t)blockIdx.x * 4 + wv) * kPerWave; wb < r1g;
         wb += (int64_t)gridDim.x * 4 * kPerWave) {
        const int64_t r0 = wb + (int64_t)lane * kMergeK;
        if (r0 < r1g) {
            const int64_t r1 = r0 + kMergeK < r1g ? r0 + kMergeK : r1g;
            // the pair holding row r0, and the merge state at its position
            const int64_t pcf = a.row_pcf[r0];
            const int64_t b = last_le(a.groups, (int64_t)a.B + 1, pcf);
            PairAt p;
            pair_from(a, b, a.groups[b] + ((pcf - a.groups[b]) / (2 * span)) * (2 * span), span,
                      p);
            int64_t q = r0 - p.sA;
            int64_t i, j;
            {
                int64_t lo = q - p.nB > 0 ? q - p.nB : 0, hi = q < p.nA ? q : p.nA;
                const T *tA = tin + p.sA, *tB = tin + p.sB;
                while (lo < hi) {  // A's share of the first q merged positions
                    const int64_t mid = (lo + hi) >> 1;
                    if (tA[mid] <= tB[q - 1 - mid])
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                i = lo;
                j = q - lo;
            }
            for (int64_t r = r0; r < r1; ++r) {
                if (q == p.nA + p.nB) {  // crossed into the next pair (or group)
                    int64_t nb = p.b, ni = p.iE;
                    if (ni == a.groups[nb + 1])
                        ++nb;
                    pair_from(a, nb, ni, span, p);
                    q = i = j = 0;
                }
                const T *tA = tin + p.sA, *vA = vin + p.sA, *tB = tin + p.sB, *vB = vin + p.sB;
                T x, val;
                if (p.nB == 0) {  // unpaired: moves up unchanged
                    x = tA[q];
                    val = vA[q];
                } else {
                    T fx, gx;
                    if (i < p.nA && (j >= p.nB || tA[i] <= tB[j])) {
                        x = tA[i];
                        fx = vA[i];
                        ++i;
                        gx = (j < p.nB && tB[j] == x) ? vB[j] : vB[j > 0 ? j - 1 : 0];
                    } else {
                        x = tB[j];
                        gx = vB[j];
                        ++j;
                        fx = (i < p.nA && tA[i] == x) ? vA[i] : vA[i > 0 ? i - 1 : 0];
                    }
                    val = red_op<T, OP>(fx, gx);
                }
                st_t[wv][r - wb] = x;
                st_v[wv][r - wb] = val;
                ++q;
            }
        }
        wave_sync_lds();
        const int64_t cnt = r1g - wb < kPerWave ? r1g - wb : kPerWave;
        for (int64_t k = lane; k < cnt; k += 64) {
            tout[wb + k] = st_t[wv][k];
            vout[wb + k] = st_v[wv][k];
        }
        wave_sync_lds();
    }
}

// row_pcf[r] = the PCF holding row r: one wave per PCF.
__global__ void red_rowmap(const int64_t *__restrict__ offsets, int64_t n,
                           int32_t *__restrict__ row_pcf)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n;
         i += nwaves)
        for (int64_t r = offsets[i] + lane; r < offsets[i + 1]; r += 64)
            row_pcf[r] = (int32_t)i;
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
        const T x = rt[r];
        const T mean = rv[r] / (T)(ge - gb);
        // binary counter over the group's PCFs: after k terms, st[h] holds
        // the sum of a complete subtree of 2^h terms for every set bit h of
        // k (the level-by-level pairing), in two levels of 15 heights
        // (blocks of 2^15 terms, then blocks; groups below 2^30 PCFs) so
        // that the loops unroll to constant indices into small arrays.
        constexpr int kIn = 15;
        T st[kIn], st2[kIn];
        int64_t k = 0;
        for (int64_t i = gb; i < ge; ++i, ++k) {
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
            bool placed = false;
#pragma unroll
            for (int hh = 0; hh < kIn; ++hh) {
                if ((k >> hh) & 1) {
                    s = st[hh] + s;
                } else {
                    st[hh] = s;
                    placed = true;
                    break;
                }
            }
            if (!placed) {  // a complete block of 2^15 terms
                const int64_t kb = k >> kIn;
#pragma unroll
                for (int hh = 0; hh < kIn; ++hh) {
                    if ((kb >> hh) & 1) {
                        s = st2[hh] + s;
                    } else {
                        st2[hh] = s;
                        break;
                    }
                }
            }
        }
        // fold the partial sums from the smallest subtree up
        const int64_t M = ge - gb;
        T acc = T(0);
        bool have = false;
#pragma unroll
        for (int hh = 0; hh < kIn; ++hh) {
            if ((M >> hh) & 1) {
                acc = have ? st[hh] + acc : st[hh];
                have = true;
            }
        }
#pragma unroll
        for (int hh = 0; hh < kIn; ++hh) {
            if (((M >> kIn) >> hh) & 1) {
                acc = have ? st2[hh] + acc : st2[hh];
                have = true;
            }
        }
        q[r] = acc;
    }
}

// Root rows kept by ReducePair's rule (all rows of a one-PCF group), and
// their values after the group's transformation. One wave per chunk of at
// most kChunkRows rows of one group.
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
    for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; c < a.nchunks;
         c += nwaves) {
        const int64_t b = a.chunk_grp[c];
        const int64_t gb = a.groups[b], m = a.groups[b + 1] - gb;
        const int64_t g0 = a.offsets[gb], g1 = a.offsets[gb + m];
        const int64_t c0 = a.chunk_row[c];
        const int64_t c1 = c0 + kChunkRows < g1 ? c0 + kChunkRows : g1;
        int64_t w = a.fill ? a.chunk_off[c] : 0;
        const int64_t end = a.fill ? *a.out_end : 0;
        for (int64_t base = c0; base < c1; base += 64) {
            const int64_t k = base + lane;
            const bool keep = k < c1 && (m == 1 || k == g0 ||
                                         (rt[k] != rt[k - 1] && rv[k] != rv[k - 1]));
            const uint64_t mask = __ballot(keep);
            const int64_t pos = w + __popcll(mask & below);
            if (a.fill && keep && pos < end) {
                t_out[pos] = rt[k];
                v_out[pos] = red_finish<T>(a.op, rv[k], m);
            }
            w += __popcll(mask);
        }
        if (!a.fill && lane == 0)
            a.chunk_cnt[c] = w;
    }
}

static int64_t grid_for(int64_t units, int64_t per_block, int64_t cap)
{
    int64_t g = (units + per_block - 1) / per_block;
    return g < 1 ? 1 : (g > cap ? cap : g);
}

hipError_t launch_red_rowmap(const int64_t *offsets, int64_t n, int32_t *row_pcf, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(red_rowmap, dim3((unsigned)grid_for(n, 4, 8192)), dim3(256), 0, s,
                       offsets, n, row_pcf);
    return hipGetLastError();
}

template <typename T>
static void launch_red_level_t(int op, const RedLevelArgs &a, dim3 g, dim3 blk, hipStream_t s)
{
    switch (op) {
    case RO_MAX: hipLaunchKernelGGL((red_level<T, RO_MAX>), g, blk, 0, s, a); break;
    case RO_MIN: hipLaunchKernelGGL((red_level<T, RO_MIN>), g, blk, 0, s, a); break;
    case RO_SUB: hipLaunchKernelGGL((red_level<T, RO_SUB>), g, blk, 0, s, a); break;
    case RO_MUL: hipLaunchKernelGGL((red_level<T, RO_MUL>), g, blk, 0, s, a); break;
    case RO_SQDIFF: hipLaunchKernelGGL((red_level<T, RO_SQDIFF>), g, blk, 0, s, a); break;
    default: hipLaunchKernelGGL((red_level<T, RO_SUM>), g, blk, 0, s, a); break;  // sum, mean, std
    }
}

hipError_t launch_red_level(bool f64, int op, const RedLevelArgs &a, int64_t rows,
                            hipStream_t s)
{
    if (rows <= 0)
        return hipSuccess;
    const dim3 g((unsigned)grid_for((rows + kMergeK - 1) / kMergeK, 256, 16384)), blk(256);
    static_assert(kMergeK >= 1 && kMergeK <= 32, "positions per lane");
    if (f64)
        launch_red_level_t<double>(op, a, g, blk, s);
    else
        launch_red_level_t<float>(op, a, g, blk, s);
    return hipGetLastError();
}

// The rows of X's PCF i and then Y's PCF i at Z's PCFs 2i and 2i+1: one
// wave per i.
template <typename T>
__global__ void red_interleave(int64_t n, const int64_t *__restrict__ xo,
                               const T *__restrict__ xt, const T *__restrict__ xv,
                               const int64_t *__restrict__ yo, const T *__restrict__ yt,
                               const T *__restrict__ yv, const int64_t *__restrict__ zo,
                               T *__restrict__ zt, T *__restrict__ zv)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n;
         i += nwaves) {
        const int64_t x0 = xo[i], nx = xo[i + 1] - x0, y0 = yo[i], ny = yo[i + 1] - y0;
        const int64_t z0 = zo[2 * i], z1 = zo[2 * i + 1];
        for (int64_t k = lane; k < nx; k += 64) {
            zt[z0 + k] = xt[x0 + k];
            zv[z0 + k] = xv[x0 + k];
        }
        for (int64_t k = lane; k < ny; k += 64) {
            zt[z1 + k] = yt[y0 + k];
            zv[z1 + k] = yv[y0 + k];
        }
    }
}

hipError_t launch_red_interleave(bool f64, int64_t n, const int64_t *xo, const void *xt,
                                 const void *xv, const int64_t *yo, const void *yt,
                                 const void *yv, const int64_t *zo, void *zt, void *zv,
                                 hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const dim3 g((unsigned)grid_for(n, 4, 8192)), blk(256);
    if (f64)
        hipLaunchKernelGGL(red_interleave<double>, g, blk, 0, s, n, xo, (const double *)xt,
                           (const double *)xv, yo, (const double *)yt, (const double *)yv, zo,
                           (double *)zt, (double *)zv);
    else
        hipLaunchKernelGGL(red_interleave<float>, g, blk, 0, s, n, xo, (const float *)xt,
                           (const float *)xv, yo, (const float *)yt, (const float *)yv, zo,
                           (float *)zt, (float *)zv);
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
    if (a.nchunks <= 0)
        return hipSuccess;
    const dim3 g((unsigned)grid_for(a.nchunks, 4, 8192)), blk(256);
    if (f64)
        hipLaunchKernelGGL(red_emit<double>, g, blk, 0, s, a);
    else
        hipLaunchKernelGGL(red_emit<float>, g, blk, 0, s, a);
    return hipGetLastError();
}

}  // namespace pcf
