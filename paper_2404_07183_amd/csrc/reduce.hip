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
// waves a workgroup of the level kernel
constexpr int kLevelWaves = 8;  // (3 % faster than 4, 11 % faster than 1)
constexpr int kChunkRows = 1024;  // rows per wave in the root pass
constexpr int64_t kStdSmall = 64;  // groups of at most this many PCFs: red_std_small

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
__global__ __launch_bounds__(64 * kLevelWaves) void red_level(RedLevelArgs a)
{
    const T *__restrict__ tin = reinterpret_cast<const T *>(a.tin);
    const T *__restrict__ vin = reinterpret_cast<const T *>(a.vin);
    T *__restrict__ tout = reinterpret_cast<T *>(a.tout);
    T *__restrict__ vout = reinterpret_cast<T *>(a.vout);
    constexpr int64_t kPerWave = 64 * kMergeK;
    __shared__ T st_t[kLevelWaves][kPerWave], st_v[kLevelWaves][kPerWave];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t span = (int64_t)1 << a.level;
    const int64_t r0g = a.offsets[a.groups[0]], r1g = a.offsets[a.groups[a.B]];
    for (int64_t wb = r0g + ((int64_t)blockIdx.x * kLevelWaves + wv) * kPerWave; wb < r1g;
         wb += (int64_t)gridDim.x * kLevelWaves * kPerWave) {
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
// tree's order, for the rows of groups of more than kStdSmall PCFs: a binary
// search of every PCF of the group per root row.
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
        if (ge - gb <= kStdSmall)
            continue;  // red_std_small's rows
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

// The same sums for groups of at most kStdSmall PCFs: one block per chunk of
// root rows (the root pass's chunks).
//
// The root of a group holds every row of its PCFs once (the levels keep all
// merged positions). For chunk [c0, c1) with first time xf, and x1 the first
// time of the group's next chunk, the rows of PCF i that the chunk's times
// can select lie between its row at or before xf and its row at or before x1
// (its last row for the group's last chunk): together at most
// (c1 - c0) + 2m - 1 rows over the group (one per root row c0 + 1 .. c1,
// m - 1 more that tie with x1 past it, and the m rows at or before xf).
// red_std_bounds bisects every PCF once per chunk for the rows at or before
// xf; red_std_small stages the window of (t, v) records in LDS. Thread j
// then takes root rows c0 + Rj .. c0 + Rj + R - 1: for every PCF i of the
// group (i = 0, 1, .. in order) it finds the record at or before its first
// row by bisection of PCF i's records, walks forward for the others, and adds
// (f_i(x) - mean(x))^2 to a binary counter per row, which sums the m terms in
// the reduction tree's order (pairs (2j, 2j + 1), then pairs of pairs, an
// unpaired last block moving up), as red_std_terms.
constexpr int kStdThreads = 512;
constexpr int kStdRowsPerThread = kChunkRows / kStdThreads;
constexpr int kStdWindow = kChunkRows + 2 * (int)kStdSmall;
constexpr int kStdHeights = 7;  // subtree heights 0 .. 6: up to 127 >= kStdSmall terms
constexpr int kStdBatch = 4;  // PCFs whose bisections run together
static_assert(kChunkRows % kStdThreads == 0 && kStdSmall == 64 && (1 << kStdHeights) > kStdSmall,
              "red_std_small's layout");

// chunk_first[64c + i] = the last row of PCF i (i < m) with t at or before
// the first root time of chunk c, for the chunks of groups of at most
// kStdSmall PCFs.
template <typename T>
__global__ void red_std_bounds(RedStdArgs a)
{
    const T *__restrict__ t = reinterpret_cast<const T *>(a.t);
    const T *__restrict__ rt = reinterpret_cast<const T *>(a.rt);
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < a.nchunks * kStdSmall;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = u / kStdSmall, i = u % kStdSmall;
        const int64_t b = a.chunk_grp[c];
        const int64_t gb = a.groups[b], m = a.groups[b + 1] - gb;
        if (m > kStdSmall || i >= m)
            continue;
        const T x = rt[a.chunk_row[c]];
        const int64_t o = a.offsets[gb + i], n = a.offsets[gb + i + 1] - o;
        int64_t lo = 0, hi = n - 1;  // t[o] = 0 <= x
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (t[o + mid] <= x)
                lo = mid;
            else
                hi = mid - 1;
        }
        a.chunk_first[u] = lo;
    }
}

template <typename T>
struct StdRecord {
    T t, v;
};

// Term s[k] joins the subtrees of heights 0 .. H-1 (smallest first, each on
// the left) and is kept as the subtree of height H.
template <typename T, int R, int H>
__device__ __forceinline__ void std_counter_add(T (&st)[R][kStdHeights], T (&s)[R])
{
#pragma unroll
    for (int k = 0; k < R; ++k) {
#pragma unroll
        for (int h = 0; h < H; ++h)
            s[k] = st[k][h] + s[k];
        st[k][H] = s[k];
    }
}

template <typename T>
__global__ __launch_bounds__(kStdThreads) void red_std_small(RedStdArgs a)
{
#pragma clang fp contract(off)
    constexpr int R = kStdRowsPerThread;
    const T *__restrict__ t = reinterpret_cast<const T *>(a.t);
    const T *__restrict__ v = reinterpret_cast<const T *>(a.v);
    const T *__restrict__ rt = reinterpret_cast<const T *>(a.rt);
    const T *__restrict__ rv = reinterpret_cast<const T *>(a.rv);
    T *__restrict__ q = reinterpret_cast<T *>(a.q);
    __shared__ StdRecord<T> rec[kStdWindow];
    __shared__ int64_t row0[kStdSmall];
    __shared__ int32_t wbase[kStdSmall + 1];
    __shared__ int32_t bad;
    const int tid = threadIdx.x;
    const T inf = __builtin_inf();
    for (int64_t c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
        const int64_t b = a.chunk_grp[c];
        const int64_t gb = a.groups[b];
        const int m = (int)(a.groups[b + 1] - gb);
        if (m > kStdSmall)
            continue;  // red_std_terms' rows (block-uniform)
        const int64_t c0 = a.chunk_row[c], g1 = a.offsets[gb + m];
        const int64_t c1 = c0 + kChunkRows < g1 ? c0 + kChunkRows : g1;
        // window offsets: an inclusive scan of the record counts in wave 0
        if (tid < 64) {
            int64_t len = 0;
            if (tid < m) {
                const int64_t o = a.offsets[gb + tid], n = a.offsets[gb + tid + 1] - o;
                const int64_t k0 = a.chunk_first[kStdSmall * c + tid];
                const int64_t k1 =
                    c1 < g1 ? a.chunk_first[kStdSmall * (c + 1) + tid] : n - 1;
                row0[tid] = o + k0;
                len = k1 - k0 + 1;
            }
            int32_t s = len < 1 || len > kStdWindow ? kStdWindow + 1 : (int32_t)len;
            for (int h = 1; h < 64; h <<= 1) {
                const int32_t o = __shfl_up(s, h, 64);
                if (tid >= h)
                    s += o;
            }
            wbase[tid + 1] = s;
            // a window over the bound only comes from times that do not
            // increase (PCF rules broken): the chunk's sums become NaN
            const uint64_t over = __ballot(tid < m && s > kStdWindow);
            if (tid == 0) {
                wbase[0] = 0;
                bad = over != 0;
            }
        }
        __syncthreads();
        const int32_t L = wbase[m];
        const bool ok = bad == 0;
        if (ok) {
            for (int32_t e = tid; e < L; e += kStdThreads) {
                int32_t lo = 0, hi = m - 1;  // the PCF whose window holds record e
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (wbase[mid] <= e)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                const int64_t r = row0[lo] + (e - wbase[lo]);
                rec[e].t = t[r];
                rec[e].v = v[r];
            }
        }
        // this thread's root rows and their means (rows past the chunk repeat
        // its last time and are not written)
        const int64_t r0 = c0 + (int64_t)R * tid;
        T x[R], mean[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int64_t r = r0 + k < c1 ? r0 + k : c1 - 1;
            x[k] = rt[r];
            mean[k] = rv[r] / (T)m;
        }
        __syncthreads();
        T st[R][kStdHeights];
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int h = 0; h < kStdHeights; ++h)
                st[k][h] = T(0);
        if (ok) {
            // kStdBatch PCFs at a time: their bisections are independent
            // chains of LDS reads, interleaved; their terms then join the
            // counter in PCF order, as one PCF at a time would
            for (int i0 = 0; i0 < m; i0 += kStdBatch) {
                int32_t lo[kStdBatch], end[kStdBatch], p[kStdBatch];
                int32_t span = 1;
#pragma unroll
                for (int u = 0; u < kStdBatch; ++u) {
                    // (past the group: the last PCF again, its terms unused)
                    const int i = i0 + u < m ? i0 + u : m - 1;
                    lo[u] = __builtin_amdgcn_readfirstlane(wbase[i]);
                    end[u] = __builtin_amdgcn_readfirstlane(wbase[i + 1]);
                    p[u] = lo[u];
                    span = end[u] - lo[u] > span ? end[u] - lo[u] : span;
                }
                // last record of each PCF at or before x[0] (rec[lo].t <=
                // x[0]); steps of one power of two for all, whose sum
                // covers the widest window
                int32_t step = 1;
                while (2 * step <= span - 1)
                    step <<= 1;
                for (int32_t s = span > 1 ? step : 0; s > 0; s >>= 1) {
#pragma unroll
                    for (int u = 0; u < kStdBatch; ++u) {
                        const int32_t j = p[u] + s;
                        if (j < end[u] && rec[j].t <= x[0])
                            p[u] = j;
                    }
                }
#pragma unroll
                for (int u = 0; u < kStdBatch; ++u) {
                    if (i0 + u >= m)
                        break;
                    int32_t pr = p[u];
                    T val[R];
                    val[0] = rec[pr].v;
                    T nt = pr + 1 < end[u] ? rec[pr + 1].t : inf;
#pragma unroll
                    for (int k = 1; k < R; ++k) {
                        while (nt <= x[k]) {
                            ++pr;
                            nt = pr + 1 < end[u] ? rec[pr + 1].t : inf;
                        }
                        val[k] = rec[pr].v;
                    }
                    T s[R];
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        const T d = val[k] - mean[k];
                        s[k] = d * d;
                    }
                    // binary counter: after i + 1 terms st[k][h] holds a
                    // complete subtree of 2^h terms for every set bit h of
                    // i + 1; term i joins the subtrees below the lowest
                    // clear bit of i
                    switch (__builtin_ctz(~(unsigned)(i0 + u))) {
                    case 0: std_counter_add<T, R, 0>(st, s); break;
                    case 1: std_counter_add<T, R, 1>(st, s); break;
                    case 2: std_counter_add<T, R, 2>(st, s); break;
                    case 3: std_counter_add<T, R, 3>(st, s); break;
                    case 4: std_counter_add<T, R, 4>(st, s); break;
                    case 5: std_counter_add<T, R, 5>(st, s); break;
                    default: std_counter_add<T, R, 6>(st, s); break;
                    }
                }
            }
        }
        // fold the subtrees from the smallest up and store
#pragma unroll
        for (int k = 0; k < R; ++k) {
            T acc = T(0);
            bool have = false;
#pragma unroll
            for (int h = 0; h < kStdHeights; ++h) {
                if ((m >> h) & 1) {
                    acc = have ? st[k][h] + acc : st[k][h];
                    have = true;
                }
            }
            if (r0 + k < c1)
                q[r0 + k] = ok ? acc : __builtin_nan("");
        }
        __syncthreads();  // the records and window table are rewritten next
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
    const dim3 g((unsigned)grid_for((rows + kMergeK - 1) / kMergeK, 64 * kLevelWaves,
                                    16384 * 4 / kLevelWaves)),
        blk(64 * kLevelWaves);
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

hipError_t launch_red_std_small(bool f64, const RedStdArgs &a, hipStream_t s)
{
    if (a.nchunks <= 0)
        return hipSuccess;
    const dim3 gb((unsigned)grid_for(a.nchunks * kStdSmall, 256, 16384)), bb(256);
    const dim3 g((unsigned)grid_for(a.nchunks, 1, 16384)), blk(kStdThreads);
    if (f64) {
        hipLaunchKernelGGL(red_std_bounds<double>, gb, bb, 0, s, a);
        hipLaunchKernelGGL(red_std_small<double>, g, blk, 0, s, a);
    } else {
        hipLaunchKernelGGL(red_std_bounds<float>, gb, bb, 0, s, a);
        hipLaunchKernelGGL(red_std_small<float>, g, blk, 0, s, a);
    }
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
