// kernels.hip -- gfx950 kernels for pairwise integrated combinations of PCFs.
//
// Method (paper, Section 3, Algorithms "IterateRectangles" and
// "CombineIntegrate"): for a pair (f, g) walk both sorted breakpoint lists
// once, left to right; every step closes one cell [x, y) of the common
// refinement with y the earlier of the two next breakpoints, adds
// h(f(x), g(x)) * (y - x) and moves the pointer(s) whose next breakpoint is
// y. The paper's pair loop is used as is; what is specific to this build:
//
//  * Breakpoint records. Row k of a PCF is packed as (t_{k+1}, v_k): the
//    value of piece k and the time where it ends; the last piece ends at a
//    finite sentinel S (largest finite value of the type), followed by
//    kPad copies of (S, v_last). A step then needs one record load, of the
//    side that advances.
//  * Ties. On equal next times only the row-side PCF advances; the column
//    side advances in the following step, whose cell has width 0 and adds
//    exactly 0. Every pair therefore takes exactly (n_f - 1) + (n_g - 1)
//    steps -- known before the loop, so work can be split exactly.
//  * Tiles and LDS. A workgroup takes a tile (row block x column block) from
//    a persistent queue, copies both blocks' records into LDS and splits the
//    tile's total step count evenly over its 1024 lanes. A lane's share may
//    start inside a pair: its starting pointers come from a merge-path
//    binary search on the pair's diagonal (the same tie order as the loop),
//    and partial sums of one pair meet in an LDS accumulator. No lane waits
//    for a longer pair, whatever the length mix.
//  * Output. Results are finished (root, unbounded-tail rule) in LDS and
//    written row by row, then transposed, both coalesced.
#include <hip/hip_runtime.h>

#include <float.h>
#include <math.h>
#include <stdint.h>

#include "common.hpp"
#include "launch.hpp"

namespace pcf {

template <typename T>
struct alignas(2 * sizeof(T)) Rec {
    T t;  // end time of the piece (sentinel for the last piece)
    T v;  // value on the piece
};

template <typename T> __device__ __forceinline__ T sentinel();
template <> __device__ __forceinline__ float sentinel<float>() { return FLT_MAX; }
template <> __device__ __forceinline__ double sentinel<double>() { return DBL_MAX; }

template <typename T, int HK>
__device__ __forceinline__ T hval(T a, T b, T p)
{
    if constexpr (HK == kAbs) {
        return fabs(a - b);
    } else if constexpr (HK == kSqr) {
        T d = a - b;
        return d * d;
    } else if constexpr (HK == kProd) {
        return a * b;
    } else {
        return pow(fabs(a - b), p);
    }
}

// ---------------------------------------------------------------------------
// Workspace access

__device__ __forceinline__ const WsHeader &hdr_of(const unsigned char *ws)
{
    return *reinterpret_cast<const WsHeader *>(ws);
}

// Largest i in [0, n) with offsets[i] <= k.
__device__ __forceinline__ int64_t pcf_of_row(const int64_t *__restrict__ offsets,
                                              int64_t n, int64_t k)
{
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Reset the tile counters (a kernel, not a memset, so that a captured
// graph replays it like any other node).
__global__ void reset_counters(unsigned char *ws)
{
    WsHeader *h = reinterpret_cast<WsHeader *>(ws);
    if (threadIdx.x < kXcds)
        h->counter[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// Pack CSR (t, v) rows into breakpoint records (see the file comment).
// Grid-stride over rows; P comes from offsets[n] on the device.
template <typename T>
__global__ void pack_records(const int64_t *__restrict__ offsets, int64_t n,
                             const T *__restrict__ t, const T *__restrict__ v,
                             unsigned char *ws)
{
    const WsHeader &h = hdr_of(ws);
    Rec<T> *rec = reinterpret_cast<Rec<T> *>(ws + h.off_rec);
    const int64_t P = offsets[n];
    const T S = sentinel<T>();
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < P;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = pcf_of_row(offsets, n, k);
        const int64_t end = offsets[i + 1];
        const int64_t at = k + i * kPad;
        const T vk = v[k];
        Rec<T> r;
        r.t = (k + 1 < end) ? t[k + 1] : S;
        r.v = vk;
        rec[at] = r;
        if (k + 1 == end) {
            r.t = S;
#pragma unroll
            for (int q = 1; q <= kPad; ++q)
                rec[at + q] = r;
        }
    }
}

// ---------------------------------------------------------------------------
// Data-contract check: per row, finite time and value, first time 0,
// strictly increasing times, last value 0. The smallest bad PCF index goes
// to the header's first_bad (initialised to INT64_MAX by the host).
template <typename T>
__global__ void validate_rows(const int64_t *__restrict__ offsets, int64_t n,
                              const T *__restrict__ t, const T *__restrict__ v,
                              unsigned char *ws)
{
    WsHeader *h = reinterpret_cast<WsHeader *>(ws);
    const int64_t P = offsets[n];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < P;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = pcf_of_row(offsets, n, k);
        const int64_t start = offsets[i], end = offsets[i + 1];
        const T tk = t[k], vk = v[k];
        bool bad = !isfinite(tk) || !isfinite(vk);
        if (k == start)
            bad = bad || (tk != T(0));
        else
            bad = bad || !(tk > t[k - 1]);
        if (k + 1 == end)
            bad = bad || (vk != T(0));
        if (bad)
            atomicMin(reinterpret_cast<unsigned long long *>(&h->first_bad),
                      (unsigned long long)i);
    }
}

// ---------------------------------------------------------------------------
// Tile kernel

struct TileShared {
    int64_t pw[kMaxPairs + 1];  // exclusive prefix of padded pair steps
    // partial sums: lane l's share of pair k lands in slot k + l (distinct
    // for all (k, l) because both the pairs and the lanes' step ranges are
    // ordered); each pair then adds its slots in lane order, so the result
    // does not depend on timing
    double part[kMaxPairs + kThreads];
    double acc[kMaxPairs];      // finished results
    int32_t rn[kMaxBlock], rb[kMaxBlock];  // row PCF rows / record base
    int32_t cn[kMaxBlock], cb[kMaxBlock];  // column PCF rows / record base
    int64_t wsum[kThreads / 64];
    int64_t tile;
    int64_t r_lo, c_lo, rrec0, crec0;
    int64_t obase, ldo, row0, col0;
    int32_t R, C, diag, mirror, global_mode, npairs;
};

constexpr int kSharedHead = (int)((sizeof(TileShared) + 255) / 256 * 256);

// Exclusive block-wide scan of one int64 per thread; returns the exclusive
// prefix and writes the total to *total (all threads).
__device__ __forceinline__ int64_t block_scan(int64_t x, int64_t *wsum,
                                              int64_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(inc, o, 64);
        if (lane >= o)
            inc += y;
    }
    if (lane == 63)
        wsum[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        int64_t s = (lane < kThreads / 64) ? wsum[lane] : 0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int64_t y = __shfl_up(s, o, 64);
            if (lane >= o)
                s += y;
        }
        if (lane < kThreads / 64)
            wsum[lane] = s;  // inclusive over waves
    }
    __syncthreads();
    const int64_t before = (wave > 0 ? wsum[wave - 1] : 0);
    *total = wsum[kThreads / 64 - 1];
    return before + inc - x;
}

// Decode a tile index into (segment, I, J); thread 0 only.
__device__ __forceinline__ void locate_tile(const WsHeader &h,
                                            const unsigned char *ws,
                                            int64_t tile, const Segment *&seg,
                                            int32_t &I, int32_t &J)
{
    const Segment *segs = reinterpret_cast<const Segment *>(ws + h.off_segs);
    int64_t lo = 0, hi = h.nseg - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (segs[mid].tile_begin <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    seg = &segs[lo];
    const int64_t t = tile - seg->tile_begin;
    if (seg->type == kSegTriangle) {
        // t = Jl (Jl + 1) / 2 + Il with 0 <= Il <= Jl
        int64_t Jl = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while (Jl * (Jl + 1) / 2 > t)
            --Jl;
        while ((Jl + 1) * (Jl + 2) / 2 <= t)
            ++Jl;
        const int64_t Il = t - Jl * (Jl + 1) / 2;
        I = seg->b0 + (int32_t)Il;
        J = seg->b0 + (int32_t)Jl;
    } else {
        const int64_t nJ = seg->c1 - seg->c0;
        I = seg->b0 + (int32_t)(t / nJ);
        J = seg->c0 + (int32_t)(t % nJ);
    }
}

// Merge-path split: number of row-side breakpoints among the first d steps
// of the pair's merge (row side first on equal times). A and B are record
// indices of the two PCFs' first records in `src`; na, nb their row counts.
template <typename T, typename Src>
__device__ __forceinline__ int32_t merge_path(Src src, int32_t A, int32_t na,
                                              int32_t B, int32_t nb, int64_t d)
{
    int64_t lo = d - (nb - 1);
    lo = lo < 0 ? 0 : lo;
    int64_t hi = d < (na - 1) ? d : (na - 1);
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const T ta = src[A + mid].t;          // breakpoint mid+1 of the row PCF
        const T tb = src[B + (d - 1 - mid)].t;  // breakpoint d-mid of the column
        if (ta <= tb)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (int32_t)lo;
}

// ---------------------------------------------------------------------------
// The merge step in CDNA assembly (LDS records, h in {|a-b|, (a-b)^2, ab}).
//
// One step: y = min(next_f, next_g); acc += h(a, b) * (y - x); then, with
// exec masked to the lanes whose row side ends first (ties included), move
// that side to its next record with one ds_read_b128/b64, and with exec
// masked to the other lanes move the column side. Written by hand because
// the compiler turns the two-armed update into register copies on both
// arms. The s_waitcnt at the end keeps the compiler's view of the loaded
// registers valid between statements. 7 VALU per step for |a-b| and ab,
// 8 for (a-b)^2.

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

template <typename T> struct RecVec;
template <> struct RecVec<double> { typedef d2v type; };
template <> struct RecVec<float> { typedef f2v type; };

#define PCF_STEP_TAIL(RD, STRIDE)                                   \
    "v_cmp_le_" #RD " vcc, %[nf], %[ng]\n\t"                      \
    "s_and_saveexec_b64 %[sv], vcc\n\t"                             \
    "v_add_u32 %[ia], " STRIDE ", %[ia]\n\t"                        \
    "ds_read_b" PCF_RECBITS_##RD " %[ra], %[ia]\n\t"               \
    "s_andn2_b64 exec, %[sv], vcc\n\t"                              \
    "v_add_u32 %[ib], " STRIDE ", %[ib]\n\t"                        \
    "ds_read_b" PCF_RECBITS_##RD " %[rb], %[ib]\n\t"               \
    "s_mov_b64 exec, %[sv]\n\t"                                     \
    "s_waitcnt lgkmcnt(0)"

#define PCF_RECBITS_f64 "128"
#define PCF_RECBITS_f32 "64"

template <typename T, int HK> struct AsmStep;

#define PCF_ASM_OPERANDS                                                      \
    : [ra] "+v"(ra), [rb] "+v"(rb), [ia] "+v"(ia), [ib] "+v"(ib),           \
      [acc] "+v"(acc), [y] "=&v"(y), [d] "=&v"(d), [dv] "=&v"(dv),          \
      [sv] "=&s"(sv)                                                        \
    : [nf] "v"(ra.x), [ng] "v"(rb.x), [a] "v"(ra.y), [b] "v"(rb.y),         \
      [x] "v"(x)                                                            \
    : "vcc", "scc", "memory"

template <> struct AsmStep<double, kAbs> {
    __device__ __forceinline__ static void run(d2v &ra, d2v &rb, uint32_t &ia,
                                               uint32_t &ib, double x, double &y,
                                               double &acc)
    {
        double d, dv;
        uint64_t sv;
        asm volatile("v_min_f64 %[y], %[nf], %[ng]\n\t"
                     "v_add_f64 %[d], %[y], -%[x]\n\t"
                     "v_add_f64 %[dv], %[a], -%[b]\n\t"
                     "v_fma_f64 %[acc], |%[dv]|, %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f64, "16")
                     PCF_ASM_OPERANDS);
    }
};
template <> struct AsmStep<double, kSqr> {
    __device__ __forceinline__ static void run(d2v &ra, d2v &rb, uint32_t &ia,
                                               uint32_t &ib, double x, double &y,
                                               double &acc)
    {
        double d, dv;
        uint64_t sv;
        asm volatile("v_min_f64 %[y], %[nf], %[ng]\n\t"
                     "v_add_f64 %[d], %[y], -%[x]\n\t"
                     "v_add_f64 %[dv], %[a], -%[b]\n\t"
                     "v_mul_f64 %[d], %[dv], %[d]\n\t"
                     "v_fma_f64 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f64, "16")
                     PCF_ASM_OPERANDS);
    }
};
template <> struct AsmStep<double, kProd> {
    __device__ __forceinline__ static void run(d2v &ra, d2v &rb, uint32_t &ia,
                                               uint32_t &ib, double x, double &y,
                                               double &acc)
    {
        double d, dv;
        uint64_t sv;
        asm volatile("v_min_f64 %[y], %[nf], %[ng]\n\t"
                     "v_add_f64 %[d], %[y], -%[x]\n\t"
                     "v_mul_f64 %[dv], %[a], %[b]\n\t"
                     "v_fma_f64 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f64, "16")
                     PCF_ASM_OPERANDS);
    }
};
template <> struct AsmStep<float, kAbs> {
    __device__ __forceinline__ static void run(f2v &ra, f2v &rb, uint32_t &ia,
                                               uint32_t &ib, float x, float &y,
                                               float &acc)
    {
        float d, dv;
        uint64_t sv;
        asm volatile("v_min_f32 %[y], %[nf], %[ng]\n\t"
                     "v_sub_f32 %[d], %[y], %[x]\n\t"
                     "v_sub_f32 %[dv], %[a], %[b]\n\t"
                     "v_fma_f32 %[acc], |%[dv]|, %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f32, "8")
                     PCF_ASM_OPERANDS);
    }
};
template <> struct AsmStep<float, kSqr> {
    __device__ __forceinline__ static void run(f2v &ra, f2v &rb, uint32_t &ia,
                                               uint32_t &ib, float x, float &y,
                                               float &acc)
    {
        float d, dv;
        uint64_t sv;
        asm volatile("v_min_f32 %[y], %[nf], %[ng]\n\t"
                     "v_sub_f32 %[d], %[y], %[x]\n\t"
                     "v_sub_f32 %[dv], %[a], %[b]\n\t"
                     "v_mul_f32 %[d], %[dv], %[d]\n\t"
                     "v_fma_f32 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f32, "8")
                     PCF_ASM_OPERANDS);
    }
};
template <> struct AsmStep<float, kProd> {
    __device__ __forceinline__ static void run(f2v &ra, f2v &rb, uint32_t &ia,
                                               uint32_t &ib, float x, float &y,
                                               float &acc)
    {
        float d, dv;
        uint64_t sv;
        asm volatile("v_min_f32 %[y], %[nf], %[ng]\n\t"
                     "v_sub_f32 %[d], %[y], %[x]\n\t"
                     "v_mul_f32 %[dv], %[a], %[b]\n\t"
                     "v_fma_f32 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f32, "8")
                     PCF_ASM_OPERANDS);
    }
};

typedef __attribute__((address_space(3))) unsigned char lds_byte;

__device__ __forceinline__ uint32_t lds_address(const void *p)
{
    return (uint32_t)(uintptr_t)(const lds_byte *)p;
}

// Starting state of steps [d, ...) of pair (A, B): record indices and x.
template <typename T, typename Src>
__device__ __forceinline__ void pair_start(Src src, int32_t A, int32_t na,
                                           int32_t B, int32_t nb, int64_t d,
                                           int32_t &ia, int32_t &ib, T &x)
{
    ia = A;
    ib = B;
    x = T(0);
    if (d > 0) {
        const int32_t i = merge_path<T>(src, A, na, B, nb, d);
        const int32_t j = (int32_t)(d - i);
        const T xa = (i > 0) ? src[A + i - 1].t : T(0);
        const T xb = (j > 0) ? src[B + j - 1].t : T(0);
        x = xa > xb ? xa : xb;
        ia = A + i;
        ib = B + j;
    }
}

// Steps [d, d + m) of pair (A, B) with records in LDS; m is a multiple of
// kStepBlock. Returns the partial sum of h * width.
template <typename T, int HK>
__device__ __forceinline__ double run_pair_lds(const Rec<T> *lrec, int32_t A,
                                               int32_t na, int32_t B,
                                               int32_t nb, int64_t d,
                                               int64_t m, T p)
{
    int32_t i0, j0;
    T x;
    pair_start<T>(lrec, A, na, B, nb, d, i0, j0, x);
    double acc = 0.0;
    if constexpr (HK == kPow) {
        int32_t ia = i0, ib = j0;
        Rec<T> ra = lrec[ia], rb = lrec[ib];
        T nf = ra.t, a = ra.v, ng = rb.t, b = rb.v;
        for (int64_t blk = 0; blk < m; blk += kStepBlock) {
            T part = T(0);
#pragma unroll
            for (int u = 0; u < kStepBlock; ++u) {
                const T y = nf <= ng ? nf : ng;
                part = fma(hval<T, HK>(a, b, p), y - x, part);
                x = y;
                if (nf <= ng) {
                    ++ia;
                    const Rec<T> r = lrec[ia];
                    nf = r.t;
                    a = r.v;
                } else {
                    ++ib;
                    const Rec<T> r = lrec[ib];
                    ng = r.t;
                    b = r.v;
                }
            }
            acc += (double)part;
        }
    } else {
        typedef typename RecVec<T>::type V;
        const V *lv = reinterpret_cast<const V *>(lrec);
        V ra = lv[i0], rb = lv[j0];
        uint32_t ia = lds_address(&lrec[i0]), ib = lds_address(&lrec[j0]);
        T x0 = x, x1;
        for (int64_t blk = 0; blk < m; blk += kStepBlock) {
            T part = T(0);
#pragma unroll
            for (int u = 0; u < kStepBlock; u += 2) {
                AsmStep<T, HK>::run(ra, rb, ia, ib, x0, x1, part);
                AsmStep<T, HK>::run(ra, rb, ia, ib, x1, x0, part);
            }
            acc += (double)part;
        }
    }
    return acc;
}

// Same from global memory (tiles too large for LDS): plain loads.
template <typename T, int HK>
__device__ __noinline__ double run_pair_global(const Rec<T> *grec, int32_t A,
                                               int32_t na, int32_t B,
                                               int32_t nb, int64_t d,
                                               int64_t m, T p)
{
    int32_t ia, ib;
    T x;
    pair_start<T>(grec, A, na, B, nb, d, ia, ib, x);
    Rec<T> ra = grec[ia], rb = grec[ib];
    T nf = ra.t, a = ra.v, ng = rb.t, b = rb.v;
    double acc = 0.0;
    for (int64_t blk = 0; blk < m; blk += kStepBlock) {
        T part = T(0);
        for (int u = 0; u < kStepBlock; ++u) {
            const T y = nf <= ng ? nf : ng;
            part = fma(hval<T, HK>(a, b, p), y - x, part);
            x = y;
            if (nf <= ng) {
                ++ia;
                const Rec<T> r = grec[ia];
                nf = r.t;
                a = r.v;
            } else {
                ++ib;
                const Rec<T> r = grec[ib];
                ng = r.t;
                b = r.v;
            }
        }
        acc += (double)part;
    }
    return acc;
}

template <typename T, int HK>
__global__ __launch_bounds__(kThreads) void pairwise_tiles(FwdArgs args)
{
    extern __shared__ __align__(16) unsigned char smem[];
    TileShared &sh = *reinterpret_cast<TileShared *>(smem);
    Rec<T> *lrec = reinterpret_cast<Rec<T> *>(smem + kSharedHead);
    const int tid = threadIdx.x;
    const unsigned char *ws = args.ws;
    const WsHeader &h = hdr_of(ws);
    const int32_t *blocks = reinterpret_cast<const int32_t *>(ws + h.off_blocks);
    const Rec<T> *grec = reinterpret_cast<const Rec<T> *>(ws + h.off_rec);
    const int64_t *offsets = args.offsets;
    const T p = (T)args.p;
    uint32_t *counter = reinterpret_cast<WsHeader *>(args.ws)->counter;

    for (;;) {
        if (tid == 0) {
            const int64_t tile = (int64_t)atomicAdd(&counter[0], 1u);
            sh.tile = tile;
            if (tile < h.ntiles) {
                const Segment *seg;
                int32_t I, J;
                locate_tile(h, ws, tile, seg, I, J);
                const int64_t r_lo = blocks[I], r_hi = blocks[I + 1];
                const int64_t c_lo = blocks[J], c_hi = blocks[J + 1];
                sh.r_lo = r_lo;
                sh.c_lo = c_lo;
                sh.R = (int32_t)(r_hi - r_lo);
                sh.C = (int32_t)(c_hi - c_lo);
                sh.diag = (seg->type == kSegTriangle && I == J) ? 1 : 0;
                sh.mirror = seg->mirror;
                sh.obase = seg->obase;
                sh.ldo = seg->ldo;
                sh.row0 = seg->row0;
                sh.col0 = seg->col0;
                sh.rrec0 = offsets[r_lo] + r_lo * kPad;
                sh.crec0 = offsets[c_lo] + c_lo * kPad;
                const int64_t rrecs = offsets[r_hi] + r_hi * kPad - sh.rrec0;
                const int64_t crecs = offsets[c_hi] + c_hi * kPad - sh.crec0;
                const int64_t need = sh.diag ? rrecs : rrecs + crecs;
                sh.global_mode = need > h.lds_records ? 1 : 0;
                sh.npairs = sh.R * sh.C;
            }
        }
        __syncthreads();
        if (sh.tile >= h.ntiles)
            break;
        const int32_t R = sh.R, C = sh.C, npairs = sh.npairs;
        const bool diag = sh.diag != 0, gmode = sh.global_mode != 0;
        const int64_t rrecs_end =
            offsets[sh.r_lo + R] + (sh.r_lo + R) * kPad - sh.rrec0;

        // block metadata: rows of each PCF and base of its records (LDS
        // index, or global index in global mode)
        if (tid < R) {
            const int64_t i = sh.r_lo + tid;
            const int64_t roff = offsets[i] + i * kPad;
            sh.rn[tid] = (int32_t)(offsets[i + 1] - offsets[i]);
            sh.rb[tid] = (int32_t)(gmode ? roff : roff - sh.rrec0);
        } else if (tid >= 64 && tid < 64 + C) {
            const int c = tid - 64;
            const int64_t j = sh.c_lo + c;
            const int64_t roff = offsets[j] + j * kPad;
            sh.cn[c] = (int32_t)(offsets[j + 1] - offsets[j]);
            sh.cb[c] = (int32_t)(gmode ? roff
                                       : (diag ? roff - sh.rrec0
                                               : rrecs_end + (roff - sh.crec0)));
        }
        // stage both blocks' records into LDS
        if (!gmode) {
            for (int64_t q = tid; q < rrecs_end; q += kThreads)
                lrec[q] = grec[sh.rrec0 + q];
            if (!diag) {
                const int64_t crecs_end =
                    offsets[sh.c_lo + C] + (sh.c_lo + C) * kPad - sh.crec0;
                for (int64_t q = tid; q < crecs_end; q += kThreads)
                    lrec[rrecs_end + q] = grec[sh.crec0 + q];
            }
        }
        __syncthreads();

        // padded step count of every pair, prefix-summed
        int64_t wp = 0;
        if (tid < npairs) {
            const int r = tid / C, c = tid - (tid / C) * C;
            bool live = true;
            if (diag)
                live = args.gram ? (r <= c) : (r < c);
            if (live) {
                const int64_t w = (int64_t)sh.rn[r] + sh.cn[c] - 2;
                wp = (w + kStepBlock - 1) / kStepBlock * kStepBlock;
            }
        }
        int64_t total;
        const int64_t excl = block_scan(wp, sh.wsum, &total);
        if (tid < npairs)
            sh.pw[tid] = excl;
        if (tid == 0)
            sh.pw[npairs] = total;
        __syncthreads();

        // this lane's share of the tile's steps
        const int64_t per = ((total + kThreads - 1) / kThreads + kStepBlock - 1) /
                            kStepBlock * kStepBlock;
        int64_t s = (int64_t)tid * per;
        const int64_t e = (s + per < total) ? s + per : total;
        if (s < e) {
            // pair containing step s: largest k with pw[k] <= s
            int32_t lo = 0, hi = npairs - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (sh.pw[mid] <= s)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            int32_t k = lo;
            int64_t d = s - sh.pw[k];
            while (s < e) {
                const int r = k / C, c = k - (k / C) * C;
                const int64_t len = sh.pw[k + 1] - sh.pw[k];
                const int64_t m = (len - d < e - s) ? len - d : e - s;
                double part;
                if (gmode)
                    part = run_pair_global<T, HK>(grec, sh.rb[r], sh.rn[r],
                                                  sh.cb[c], sh.cn[c], d, m, p);
                else
                    part = run_pair_lds<T, HK>(lrec, sh.rb[r], sh.rn[r],
                                               sh.cb[c], sh.cn[c], d, m, p);
                sh.part[k + tid] = part;
                s += m;
                d = 0;
                ++k;
                while (k < npairs && sh.pw[k + 1] == sh.pw[k])
                    ++k;
            }
        }
        __syncthreads();

        // finish: unbounded-tail rule, root; write (i, j) row-major
        const Rec<T> *src = gmode ? grec : lrec;
        for (int k = tid; k < npairs; k += kThreads) {
            const int r = k / C, c = k - (k / C) * C;
            if (diag && r > c)
                continue;
            double val = 0.0;
            const int64_t b0 = sh.pw[k], b1 = sh.pw[k + 1];
            if (b1 > b0) {
                const int64_t l0 = b0 / per, l1 = (b1 - 1) / per;
                for (int64_t l = l0; l <= l1; ++l)
                    val += sh.part[k + l];
            }
            const T la = src[sh.rb[r] + sh.rn[r] - 1].v;
            const T lb = src[sh.cb[c] + sh.cn[c] - 1].v;
            const T ht = hval<T, HK>(la, lb, p);
            if (ht != T(0))
                val = ht > T(0) ? INFINITY : -INFINITY;
            if (args.root == kRootSqrt)
                val = sqrt(val);
            else if (args.root == kRootPow)
                val = pow(val, args.inv_p);
            sh.acc[k] = val;
            const int64_t i = sh.r_lo + r, j = sh.c_lo + c;
            T *out = reinterpret_cast<T *>(args.out);
            out[sh.obase + (i - sh.row0) * sh.ldo + (j - sh.col0)] = (T)val;
        }
        if (sh.mirror) {
            __syncthreads();
            for (int q = tid; q < npairs; q += kThreads) {
                const int c = q / R, r = q - (q / R) * R;
                if (diag && r >= c)
                    continue;
                const double val = sh.acc[r * C + c];
                const int64_t i = sh.r_lo + r, j = sh.c_lo + c;
                T *out = reinterpret_cast<T *>(args.out);
                out[sh.obase + (j - sh.row0) * sh.ldo + (i - sh.col0)] = (T)val;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the C-ABI layer).

size_t tile_shared_bytes(int rec_bytes, bool backward)
{
    const int per = rec_bytes + (backward ? 16 : 0);
    return (size_t)kSharedHead + (size_t)(kLdsRecordBytes / per) * per;
}

template <typename T>
hipError_t launch_pack(const int64_t *offsets, int64_t n, const void *t,
                       const void *v, unsigned char *ws, int64_t P,
                       hipStream_t s)
{
    if (P <= 0)
        return hipSuccess;
    int64_t blocks = (P + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(pack_records<T>, dim3((unsigned)blocks), dim3(256), 0, s,
                       offsets, n, (const T *)t, (const T *)v, ws);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_validate(const int64_t *offsets, int64_t n, const void *t,
                           const void *v, unsigned char *ws, int64_t P,
                           hipStream_t s)
{
    if (P <= 0)
        return hipSuccess;
    int64_t blocks = (P + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(validate_rows<T>, dim3((unsigned)blocks), dim3(256), 0,
                       s, offsets, n, (const T *)t, (const T *)v, ws);
    return hipGetLastError();
}

hipError_t launch_reset(unsigned char *ws, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, ws);
    return hipGetLastError();
}

template <typename T, int HK>
static hipError_t launch_fwd_t(const FwdArgs &a, int grid, hipStream_t s)
{
    const size_t shm = tile_shared_bytes((int)sizeof(Rec<T>), false);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&pairwise_tiles<T, HK>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess)
            return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((pairwise_tiles<T, HK>), dim3(grid), dim3(kThreads), shm,
                       s, a);
    return hipGetLastError();
}

hipError_t launch_forward(bool f64, int hk, const FwdArgs &a, int grid,
                          hipStream_t s)
{
    if (f64) {
        switch (hk) {
        case kAbs: return launch_fwd_t<double, kAbs>(a, grid, s);
        case kSqr: return launch_fwd_t<double, kSqr>(a, grid, s);
        case kProd: return launch_fwd_t<double, kProd>(a, grid, s);
        default: return launch_fwd_t<double, kPow>(a, grid, s);
        }
    } else {
        switch (hk) {
        case kAbs: return launch_fwd_t<float, kAbs>(a, grid, s);
        case kSqr: return launch_fwd_t<float, kSqr>(a, grid, s);
        case kProd: return launch_fwd_t<float, kProd>(a, grid, s);
        default: return launch_fwd_t<float, kPow>(a, grid, s);
        }
    }
}

template hipError_t launch_pack<float>(const int64_t *, int64_t, const void *,
                                       const void *, unsigned char *, int64_t,
                                       hipStream_t);
template hipError_t launch_pack<double>(const int64_t *, int64_t, const void *,
                                        const void *, unsigned char *, int64_t,
                                        hipStream_t);
template hipError_t launch_validate<float>(const int64_t *, int64_t,
                                           const void *, const void *,
                                           unsigned char *, int64_t,
                                           hipStream_t);
template hipError_t launch_validate<double>(const int64_t *, int64_t,
                                            const void *, const void *,
                                            unsigned char *, int64_t,
                                            hipStream_t);

}  // namespace pcf
