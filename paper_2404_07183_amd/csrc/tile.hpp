// tile.hpp -- device-side pieces shared by the forward and adjoint tile
// kernels: breakpoint records, the tile queue, LDS staging, the per-pair
// step prefix and the merge-path split (see kernels.hip for the method).
#pragma once

#include <hip/hip_runtime.h>

#include <float.h>
#include <math.h>
#include <stdint.h>

#include <utility>

#include "common.hpp"
#include "launch.hpp"
#include "pow64.hpp"

namespace pcf {

template <typename T>
struct alignas(2 * sizeof(T)) Rec {
    T t;  // end time of the piece (sentinel for the last piece)
    T v;  // value on the piece
};

template <typename T> __device__ __forceinline__ T sentinel();
template <> __device__ __forceinline__ float sentinel<float>() { return FLT_MAX; }
template <> __device__ __forceinline__ double sentinel<double>() { return DBL_MAX; }

// x^k for a launch-uniform integer k >= 1, by squaring.
template <typename T>
__device__ __forceinline__ T ipow(T x, int k)
{
    T r = (k & 1) ? x : T(1);
    for (k >>= 1; k > 0; k >>= 1) {
        x *= x;
        if (k & 1)
            r *= x;
    }
    return r;
}

// x^p for p = k + 1/2 (k >= 0, launch-uniform): x^k by squaring, times
// sqrt(x).
template <typename T>
__device__ __forceinline__ T pow_half(T x, T p)
{
    const int k = (int)p;
    return k > 0 ? ipow(x, k) * sqrt(x) : sqrt(x);
}

// x^p = 2^(p log2 x) for any other p: FP32 by the hardware base-2 log and
// exp (v_log_f32, v_exp_f32; relative error a few ulps times |p log2 x|,
// x = 0 gives 0), FP64 by the series of pow64.hpp.
__device__ __forceinline__ float pow_any(float x, float p)
{
    return __builtin_amdgcn_exp2f(p * __builtin_amdgcn_logf(x));
}
__device__ __forceinline__ double pow_any(double x, double p) { return pow_series(x, p); }

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
    } else if constexpr (HK == kPowHalf) {
        return pow_half(fabs(a - b), p);
    } else if constexpr (HK == kPowInt) {
        return ipow(fabs(a - b), (int)p);
    } else {
        return pow_any(fabs(a - b), p);
    }
}

// ---------------------------------------------------------------------------
// Per-phase cycle counters of the tile loop, compiled in only with
// -DPCF_PHASE_TIMING (a measurement build; the library's own build has empty
// inline members). The shader-clock counter is read at each phase boundary;
// the first lane of every wave adds its sums to g_phase_cycles at the end
// (slots 16 * wave + phase, tiles at + 8, steps at + 9, pair-switch cycles
// and count at + 10 and + 11; wave 15 holds the queue lane).
enum Phase : int {
    kPhaseScan = 0, kPhaseStart = 1, kPhaseMerge = 2, kPhaseMergeWait = 3,
    kPhaseStageIssue = 4, kPhaseFinish = 5, kPhaseStageStore = 6, kPhaseAdvance = 7
};
#ifdef PCF_PHASE_TIMING
__device__ unsigned long long g_phase_cycles[16 * 16];
struct PhaseClock {
    unsigned long long acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long last = 0, tiles = 0, steps = 0, sw = 0, swn = 0;
    unsigned long long subacc[3] = {0, 0, 0};
    // time from the last phase boundary to sub-phase point q of the scan
    __device__ __forceinline__ void sub(int q) { subacc[q] += now() - last; }
    __device__ __forceinline__ unsigned long long now() const
    {
        return __builtin_readcyclecounter();
    }
    // time spent in a wave's pair-switch branch, and how often it is taken
    __device__ __forceinline__ void sw_add(unsigned long long t0, bool taken)
    {
        sw += now() - t0;
        swn += taken ? 1 : 0;
    }
    __device__ __forceinline__ void mark(int q)
    {
        const unsigned long long now = __builtin_readcyclecounter();
        if (q >= 0)
            acc[q] += now - last;
        last = now;
    }
    __device__ __forceinline__ void tile(int64_t s)
    {
        ++tiles;
        steps += (unsigned long long)s;
    }
    __device__ __forceinline__ void flush(int who)
    {
        if (who < 0)
            return;
        for (int q = 0; q < 8; ++q)
            atomicAdd(&g_phase_cycles[16 * who + q], acc[q]);
        atomicAdd(&g_phase_cycles[16 * who + 8], tiles);
        atomicAdd(&g_phase_cycles[16 * who + 9], steps);
        atomicAdd(&g_phase_cycles[16 * who + 10], sw);
        atomicAdd(&g_phase_cycles[16 * who + 11], swn);
        for (int q = 0; q < 3; ++q)
            atomicAdd(&g_phase_cycles[16 * who + 12 + q], subacc[q]);
    }
};
#else
struct PhaseClock {
    __device__ __forceinline__ void sub(int) {}
    __device__ __forceinline__ unsigned long long now() const { return 0; }
    __device__ __forceinline__ void sw_add(unsigned long long, bool) {}
    __device__ __forceinline__ void mark(int) {}
    __device__ __forceinline__ void tile(int64_t) {}
    __device__ __forceinline__ void flush(int) {}
};
#endif

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
// Tile kernel

// A decoded tile: which blocks, where their records are, where the results
// go. Written by the queue lane, read by all threads from LDS.
struct TileDesc {
    int64_t tile;          // >= ntiles: the queue is empty
    int64_t r_lo, c_lo;    // first PCF of the row / column block
    int64_t rrec0, crec0;  // first global record of the row / column block
    int64_t rrecs, crecs;  // records of the row / column block
    int64_t obase, ldo, row0, col0;  // output mapping of the segment
    int32_t R, C, diag, mirror, global_mode;
    int32_t cmag;          // floor(2^16 / C) + 1 (see div_by_c)
};

template <int PartSlots> struct TileSharedT {
    // exclusive prefix of padded pair steps, 32-bit; a tile whose step
    // total may reach 2^30 (only global-mode tiles) keeps it in 64 bits at
    // the start of the LDS record area instead (pw_wide; see pw_at)
    int32_t pw[kMaxPairs + 1];
    // partial sums: lane l's share of pair k lands in slot k + l (distinct
    // for all (k, l) because both the pairs and the lanes' step ranges are
    // ordered); each pair then adds its slots in lane order, from the lane
    // of its first step to the lane of its last (lane_of), so the result
    // does not depend on timing
    double part[PartSlots];
    int16_t pairof[kThreads];  // pair holding the first step of each lane
    int32_t rn[kMaxBlock], rb[kMaxBlock];  // row PCF rows / record base
    int32_t cn[kMaxBlock], cb[kMaxBlock];  // column PCF rows / record base
    double rlast[kMaxBlock], clast[kMaxBlock];  // last values (tail rule)
    int64_t wsum[kThreads / 64];
    TileDesc desc[3];  // ring of tile descriptors (see TileLoop)
    int64_t gper[4];   // steps per lane of each wave group (see LaneSplit)
    int64_t gbase[5];  // first step of each wave group
    int32_t npairs;
    int32_t cmag;      // the current tile's cmag (see div_by_c)
    int32_t pw_wide;   // the step prefix is the 64-bit one in the record area
};
// The forward kernels' tile state: partial-sum slots for every (pair, lane)
// combination a tile can produce (see part).
using TileShared = TileSharedT<kMaxPairs + kThreads>;

constexpr int kSharedHead = (int)((sizeof(TileShared) + 255) / 256 * 256);
static_assert(kSharedHead + kLdsRecordBytes <= 160 * 1024 / kWgPerCu,
              "the tile workgroups of a CU must fit its 160 KiB of LDS");

// k / C for 0 <= k < 2048 and 1 <= C <= 32, by a multiply: with
// m = floor(2^16 / C) + 1, k m / 2^16 exceeds k / C by less than
// k / 2^16 < 1/32 <= 1/C, which cannot carry it past the next integer (the
// fractional part of k / C is at most 1 - 1/C).
static_assert(kMaxBlock <= 32 && kMaxPairs <= 2048, "div_by_c range");
__device__ __forceinline__ int32_t div_by_c(int32_t k, int32_t cmag)
{
    return (int32_t)(((uint32_t)k * (uint32_t)cmag) >> 16);
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, not for its global stores (no thread of the workgroup reads
// the output back), so writing a tile's results does not stall the next.
__device__ __forceinline__ void sync_lds()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Exclusive block-wide scan of one integer per thread; returns the exclusive
// prefix and the block total. Two barriers. `wsum` holds kThreads / 64
// values of type I.
template <typename I>
__device__ __forceinline__ I block_scan(I x, I *wsum, I *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    I inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const I y = __shfl_up(inc, o, 64);
        if (lane >= o)
            inc += y;
    }
    if (lane == 63)
        wsum[wave] = inc;
    sync_lds();
    if (wave == 0) {
        I v = (lane < kThreads / 64) ? wsum[lane] : I(0);
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const I y = __shfl_up(v, o, 64);
            if (lane >= o)
                v += y;
        }
        if (lane < kThreads / 64)
            wsum[lane] = v;  // inclusive over waves
    }
    sync_lds();
    const I before = (wave > 0 ? wsum[wave - 1] : I(0));
    *total = wsum[kThreads / 64 - 1];
    return before + inc - x;
}

// The 32-bit scan: the wave's inclusive scan with DPP row shifts (1, 2, 4, 8
// within rows of 16 lanes) and row broadcasts (lane 15 into the next row,
// lane 31 into rows 2 and 3), lanes without a source adding 0; then one
// barrier, after which every wave adds the totals of the waves before it.
template <>
__device__ __forceinline__ int32_t block_scan<int32_t>(int32_t x, int32_t *wsum,
                                                       int32_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t v = x;
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    if (lane == 63)
        wsum[wave] = v;
    sync_lds();
    // the sixteen wave totals, scanned again inside each row of 16 lanes
    static_assert(kThreads == 1024, "one wave total per lane of a DPP row");
    int32_t w = wsum[lane & 15];
    w += __builtin_amdgcn_update_dpp(0, w, 0x111, 0xf, 0xf, false);
    w += __builtin_amdgcn_update_dpp(0, w, 0x112, 0xf, 0xf, false);
    w += __builtin_amdgcn_update_dpp(0, w, 0x114, 0xf, 0xf, false);
    w += __builtin_amdgcn_update_dpp(0, w, 0x118, 0xf, 0xf, false);
    *total = __builtin_amdgcn_readlane(w, 15);
    const int sw = __builtin_amdgcn_readfirstlane(wave);
    const int32_t before = __builtin_amdgcn_readlane(w, sw > 0 ? sw - 1 : 0);
    return (sw > 0 ? before : 0) + v - x;
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
                                              int32_t B, int32_t nb, int32_t d)
{
    // 32-bit: d is below a pair's step count, which stays below 2^31
    int32_t lo = d - (nb - 1);
    lo = lo < 0 ? 0 : lo;
    int32_t hi = d < (na - 1) ? d : (na - 1);
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        const T ta = src[A + mid].t;          // breakpoint mid+1 of the row PCF
        const T tb = src[B + (d - 1 - mid)].t;  // breakpoint d-mid of the column
        if (ta <= tb)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

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
        const int32_t i = merge_path<T>(src, A, na, B, nb, (int32_t)d);
        const int32_t j = (int32_t)d - i;
        const T xa = (i > 0) ? src[A + i - 1].t : T(0);
        const T xb = (j > 0) ? src[B + j - 1].t : T(0);
        x = xa > xb ? xa : xb;
        ia = A + i;
        ib = B + j;
    }
}

// The lane that takes tickets from the tile queue and decodes the next tile:
// first lane of the last wave, which has no finishing work while a tile has
// at most kThreads - 64 pairs.
constexpr int kQueueLane = kThreads - 64;

// Takes the next ticket from the tile queue. The ticket stays 32-bit until
// it is decoded, so that no instruction reads the returned value (and waits
// for it) before the decode, after the merge work.
__device__ __forceinline__ uint32_t tile_ticket(const unsigned char *ws)
{
    uint32_t *counter =
        const_cast<uint32_t *>(reinterpret_cast<const WsHeader *>(ws)->counter);
    return atomicAdd(&counter[0], 1u);
}

// Decodes ticket `tile` into d (one lane).
__device__ __forceinline__ void tile_decode(TileDesc &d, int64_t tile,
                                            const unsigned char *ws,
                                            const int64_t *offsets)
{
    const WsHeader &h = hdr_of(ws);
    d.tile = tile;
    if (tile >= h.ntiles)
        return;
    const int32_t *blocks = reinterpret_cast<const int32_t *>(ws + h.off_blocks);
    const Segment *seg;
    int32_t I, J;
    locate_tile(h, ws, tile, seg, I, J);
    const int64_t r_lo = blocks[I], r_hi = blocks[I + 1];
    const int64_t c_lo = blocks[J], c_hi = blocks[J + 1];
    d.r_lo = r_lo;
    d.c_lo = c_lo;
    d.R = (int32_t)(r_hi - r_lo);
    d.C = (int32_t)(c_hi - c_lo);
    d.cmag = (1 << 16) / d.C + 1;
    d.diag = (seg->type == kSegTriangle && I == J) ? 1 : 0;
    d.mirror = seg->mirror;
    d.obase = seg->obase;
    d.ldo = seg->ldo;
    d.row0 = seg->row0;
    d.col0 = seg->col0;
    d.rrec0 = offsets[r_lo] + r_lo * kPad;
    d.crec0 = offsets[c_lo] + c_lo * kPad;
    d.rrecs = offsets[r_hi] + r_hi * kPad - d.rrec0;
    d.crecs = offsets[c_hi] + c_hi * kPad - d.crec0;
    const int64_t need = d.diag ? d.rrecs : d.rrecs + d.crecs;
    d.global_mode = need > h.lds_records ? 1 : 0;
}

// Records each thread stages, so that one pass moves a full LDS record area.
template <typename T>
constexpr int stage_unroll()
{
    return (int)((kLdsRecordBytes + kThreads * (int)sizeof(Rec<T>) - 1) /
                 (kThreads * (int)sizeof(Rec<T>)));
}

// One thread's part of a tile's staging, held in registers between the
// loads (issued early) and the LDS stores: up to stage_unroll() records and,
// for threads [0, R) and [64, 64 + C), one PCF's offsets.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
template <typename T> struct RecVec;
template <> struct RecVec<double> { typedef d2v type; };
template <> struct RecVec<float> { typedef f2v type; };

// v_min / v_max without the quieting of signalling NaNs that fmin/fmax
// would add (the data contract excludes NaN).
__device__ __forceinline__ double min_raw(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float min_raw(float a, float b)
{
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double max_raw(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float max_raw(float a, float b)
{
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Record addresses of a chain's two pieces. Global mode keeps both
// pointers. LDS mode keeps one 32-bit address and a sum instead: every step
// loads exactly one record, the successor of the piece that ends, so
// addr(P) + addr(Q) grows by one record per step. With S that sum at the
// start of a block of kStepBlock steps and q = addr(P) - k * rec at step k
// of the block (rec = record bytes), addr(Q) - k * rec = |S - q| - k * rec
// (one v_sad_u32); the ending piece's address minus k * rec is a select of
// the two and becomes the next q, and its successor is read at that plus
// (k + 1) * rec, a constant offset of the LDS read. Two VALU instructions
// per step instead of three.
template <typename T> struct LdsWalk {
    typedef typename RecVec<T>::type V;
    typedef const __attribute__((address_space(3))) V *ptr;
    static constexpr uint32_t kRec = sizeof(Rec<T>);
    uint32_t q, S;

    __device__ __forceinline__ void set(const Rec<T> *base, int32_t iP, int32_t iQ)
    {
        q = lds_address(base + iP);
        S = q + lds_address(base + iQ);
    }
    __device__ __forceinline__ static V at(const Rec<T> *base, int32_t i)
    {
        return *(ptr)(size_t)lds_address(base + i);
    }
    template <int K>
    __device__ __forceinline__ V advance(bool p_ends)
    {
        uint32_t b;
        asm("v_sad_u32 %0, %1, %2, %3"
            : "=v"(b)
            : "v"(S), "v"(q), "s"((uint32_t)(0u - K * kRec)));
        const uint32_t m = p_ends ? q : b;
        q = m;
        return *(ptr)(size_t)(m + (uint32_t)(K + 1) * kRec);
    }
    __device__ __forceinline__ void end_block()
    {
        q += kStepBlock * kRec;
        S += kStepBlock * kRec;
    }
};

// Direct staging (`Direct`, FP64 records only) moves records straight from
// global memory to LDS (global_load_lds_dwordx4: each lane's record lands at
// the wave's LDS base plus 16 bytes per lane), with no register round trip
// or LDS store instructions. The compiler then makes every later LDS read
// wait for those loads unless it can tell the tile state apart (a separate
// LDS object), so it pays where staging is not overlapped with other LDS
// work (the adjoint); the forward kernel stages through registers, with the
// loads in flight while it finishes the current tile.
template <typename T, bool Direct, int U = stage_unroll<T>()>
struct StageRegs {
    static_assert(!Direct || sizeof(Rec<T>) == 16, "direct staging moves 16-byte records");
    typename RecVec<T>::type r[Direct ? 1 : U];
    int64_t m0, m1;
};

// Loads of tile d's staging: its records (row block, then column block
// unless diagonal; none in global mode) and the block metadata.
template <typename T, bool Direct, int U = stage_unroll<T>()>
__device__ __forceinline__ void stage_load(StageRegs<T, Direct, U> &g, const TileDesc &d,
                                           const Rec<T> *grec,
                                           const int64_t *offsets, Rec<T> *lrec)
{
    typedef typename RecVec<T>::type V;
    const int tid = threadIdx.x;
    const int64_t rrecs = d.rrecs, rrec0 = d.rrec0, crec0 = d.crec0;
    const int64_t total = d.global_mode ? 0 : (d.diag ? rrecs : rrecs + d.crecs);
    if (total > 0) {
        // a tile's LDS records number less than 2^31, so 32-bit indices
        const V *rbase = reinterpret_cast<const V *>(grec) + rrec0;
        const V *cbase = reinterpret_cast<const V *>(grec) + (crec0 - rrecs);
        const int32_t tot = (int32_t)total, nr = (int32_t)rrecs;
        if constexpr (Direct) {
            // whole waves past the end issue nothing; in the last wave the
            // lanes past the end reload record 0 into slots below the next
            // multiple of 64 records, inside the record area
            const int32_t wbase = __builtin_amdgcn_readfirstlane(tid & ~63);
            // not unrolled: one load instruction, which the compiler's
            // tracking of direct-to-LDS loads can tell apart from the tile
            // state (so reads of the latter do not wait for these loads)
#pragma unroll 1
            for (int u = 0; u < U; ++u) {
                const int32_t q0 = wbase + u * kThreads;
                if (q0 < tot) {
                    int32_t q = tid + u * kThreads;
                    q = q < tot ? q : 0;
                    __builtin_amdgcn_global_load_lds(
                        (const void *)((q < nr ? rbase : cbase) + q),
                        (void *)(reinterpret_cast<V *>(lrec) + q0), 16, 0, 0);
                }
            }
        } else {
            // unconditional loads (indices past the end read record 0 of
            // the tile again), so that the values stay in registers
#pragma unroll
            for (int u = 0; u < U; ++u) {
                int32_t q = tid + u * kThreads;
                q = q < tot ? q : 0;
                g.r[u] = (q < nr ? rbase : cbase)[q];
            }
        }
    }
    const bool mrow = tid < d.R;
    const bool mcol = tid >= 64 && tid < 64 + d.C;
    if (mrow || mcol) {
        const int64_t i = mrow ? d.r_lo + tid : d.c_lo + (tid - 64);
        g.m0 = offsets[i];
        g.m1 = offsets[i + 1];
    }
}

// LDS stores of tile d's staging (after stage_load on the same thread).
template <typename T, bool Direct, int U = stage_unroll<T>(), typename Sh>
__device__ __forceinline__ void stage_store(Sh &sh, const StageRegs<T, Direct, U> &g,
                                            const TileDesc &d, Rec<T> *lrec)
{
    const int tid = threadIdx.x;
    const int64_t rrecs = d.rrecs;
    const int64_t total = d.global_mode ? 0 : (d.diag ? rrecs : rrecs + d.crecs);
    typedef typename RecVec<T>::type V;
    V *lv = reinterpret_cast<V *>(lrec);
    const int32_t tot = (int32_t)total;
    if constexpr (Direct) {
        // the direct loads have landed (the barrier that follows publishes
        // them to the workgroup)
        (void)lv;
        (void)tot;
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t q = tid + u * kThreads;
            if (q < tot)
                lv[q] = g.r[u];
        }
    }
    const bool mrow = tid < d.R;
    const bool mcol = tid >= 64 && tid < 64 + d.C;
    if (mrow || mcol) {
        const bool gmode = d.global_mode != 0;
        const int64_t i = mrow ? d.r_lo + tid : d.c_lo + (tid - 64);
        const int64_t roff = g.m0 + i * kPad;
        const int32_t n = (int32_t)(g.m1 - g.m0);
        if (mrow) {
            sh.rn[tid] = n;
            sh.rb[tid] = (int32_t)(gmode ? roff : roff - d.rrec0);
        } else {
            const int c = tid - 64;
            sh.cn[c] = n;
            sh.cb[c] = (int32_t)(gmode ? roff
                                       : (d.diag ? roff - d.rrec0
                                                 : rrecs + (roff - d.crec0)));
        }
    }
}

// Split of a tile's steps over its lanes. The waves of a workgroup form four
// age groups (waves 4g..4g+3, one per SIMD); each SIMD issues the older of
// its waves first, so equal runs would leave the youngest group finishing
// last while the others wait. Group g's lanes get runs in proportion to
// kGroupWeight[g] (their measured issue share), so that all groups finish
// together. Runs are multiples of kStepBlock (pair step counts are too, so a
// block never straddles two pairs) and lie in [gbase[g], gbase[g + 1]) for
// group g, lane by lane; the last runs of the tile may be short or empty.
constexpr int kGroups = kThreads / 256;
constexpr int kGroupLanes = 256;
// Weights measured on MI355X (per-wave completion times of equal runs):
// forward FP64 records, forward FP32 records, the adjoint (FP64; its waves
// differ more in speed, older waves winning the LDS atomics and issue).
constexpr int kWeightsF64 = 0, kWeightsF32 = 1, kWeightsAdjoint = 2;
constexpr int64_t kGroupWeights[3][4] = {{66, 61, 53, 38}, {64, 60, 55, 45}, {83, 62, 44, 29}};
template <typename T>
constexpr int forward_weights()
{
    return sizeof(T) == 4 ? kWeightsF32 : kWeightsF64;
}
template <int WS>
__device__ __forceinline__ int64_t group_weight(int g)
{
    return kGroupWeights[WS][g];
}
template <int WS>
constexpr int64_t weight_sum()
{
    int64_t w = 0;
    for (int g = 0; g < kGroups; ++g)
        w += kGroupWeights[WS][g];
    return w;
}

// a / b for 0 <= a < 2^30, 8 <= b < 2^30 and a / b < 2^10: a float
// reciprocal estimate (off by at most one at these ratios), corrected
__device__ __forceinline__ int32_t quot_small(int32_t a, int32_t b)
{
    int32_t j = (int32_t)((float)a * __builtin_amdgcn_rcpf((float)b));
    const int32_t r = a - j * b;
    j += (r >= b ? 1 : 0) - (r < 0 ? 1 : 0);
    return j;
}

template <int WS>
struct LaneSplit {
    int64_t per[kGroups], base[kGroups + 1];

    __device__ __forceinline__ void make(int64_t total)
    {
        // groups before the last: their share rounded to whole blocks; the
        // last group takes the rest (rounded up)
        constexpr int64_t kUnit = kGroupLanes * weight_sum<WS>();
        base[0] = 0;
#pragma unroll
        for (int g = 0; g < kGroups; ++g) {
            int64_t p;
            if (g + 1 < kGroups) {
                p = (total * group_weight<WS>(g) + kUnit * kStepBlock / 2) /
                    (kUnit * kStepBlock) * kStepBlock;
            } else {
                const int64_t rest = total - base[g];
                p = ((rest > 0 ? rest : 0) + kGroupLanes - 1) / kGroupLanes;
                p = (p + kStepBlock - 1) / kStepBlock * kStepBlock;
            }
            per[g] = p < kStepBlock ? kStepBlock : p;
            base[g + 1] = base[g] + kGroupLanes * per[g];
        }
    }
    // make() for totals below 2^30, with the divisions by constants done
    // in FP64 (the same instructions on every lane, so the same split)
    __device__ __forceinline__ void make_small(int32_t total)
    {
        constexpr double kInv = 1.0 / (double)(kGroupLanes * weight_sum<WS>() * kStepBlock);
        int32_t b = 0;
        base[0] = 0;
#pragma unroll
        for (int g = 0; g < kGroups; ++g) {
            int32_t p;
            if (g + 1 < kGroups) {
                p = (int32_t)rint((double)total * (double)group_weight<WS>(g) * kInv) *
                    kStepBlock;
            } else {
                const int32_t rest = total - b > 0 ? total - b : 0;
                p = (rest + kGroupLanes - 1) / kGroupLanes;
                p = (p + kStepBlock - 1) & ~(kStepBlock - 1);
            }
            p = p < kStepBlock ? kStepBlock : p;
            per[g] = p;
            b += kGroupLanes * p;
            base[g + 1] = b;
        }
    }
    // a / b for 0 <= a, 0 < b, in 32 bits when both fit
    __device__ __forceinline__ static int32_t quot(int64_t a, int64_t b)
    {
        if (a < ((int64_t)1 << 31) && b < ((int64_t)1 << 31))
            return (int32_t)((uint32_t)a / (uint32_t)b);
        return (int32_t)(a / b);
    }
};

// Entry k of the tile's step prefix (pw64: the LDS record area).
template <typename Sh>
__device__ __forceinline__ int64_t pw_at(const Sh &sh, const int64_t *pw64, int k)
{
    return sh.pw_wide ? pw64[k] : (int64_t)sh.pw[k];
}

// The lane whose run holds step `step` of the tile (the inverse of
// lane_steps).
template <typename Sh>
__device__ __forceinline__ int32_t lane_of(const Sh &sh, int64_t step)
{
    const int g = (step >= sh.gbase[1] ? 1 : 0) + (step >= sh.gbase[2] ? 1 : 0) +
                  (step >= sh.gbase[3] ? 1 : 0);
    const int64_t a = step - sh.gbase[g], b = sh.gper[g];
    int32_t j;
    if (!sh.pw_wide)
        j = quot_small((int32_t)a, (int32_t)b);
    else
        j = (int32_t)(a / b);
    return g * kGroupLanes + j;
}

// Steps [s, e) of lane `lane` (e <= s when it has none).
template <typename Sh>
__device__ __forceinline__ void lane_steps(const Sh &sh, int lane,
                                           int64_t total, int64_t &s, int64_t &e)
{
    const int g = lane / kGroupLanes;
    s = sh.gbase[g] + (int64_t)(lane - g * kGroupLanes) * sh.gper[g];
    e = s + sh.gper[g];
    e = e < total ? e : total;
}


// an LDS tile's step total stays below 2^30, so only global-mode tiles (which
// leave the record area unused) take the 64-bit prefix
static_assert((int64_t)kMaxBlock * (kLdsRecordBytes / 8) + 8 * (int64_t)kMaxPairs <
                  ((int64_t)1 << 30),
              "LDS tiles scan in 32 bits");

// Padded step count of every pair of tile d, prefix-summed into sh.pw, or
// into pw64 (the LDS record area, unused by global-mode tiles, the only ones
// whose total may reach 2^30)
// (diagonal tiles give work to pairs r < c, and to r == c when `gram`);
// the split of the total over the lanes (sh.gper, sh.gbase: LaneSplit) and,
// for each lane, the pair holding its first step (sh.pairof); the last value
// of every PCF of the tile (sh.rlast, clast),
// read from `src` (the LDS records, or the packed records in global mode).
// Needs the staged tile; ends with a barrier.
template <typename T, int WS = forward_weights<T>(), typename Sh>
__device__ __forceinline__ void tile_scan(Sh &sh, const TileDesc &d,
                                          int gram, const Rec<T> *src, int64_t *pw64,
                                          PhaseClock &pc)
{
    const int tid = threadIdx.x;
    if (tid < d.R)
        sh.rlast[tid] = (double)src[sh.rb[tid] + sh.rn[tid] - 1].v;
    else if (tid >= 64 && tid < 64 + d.C)
        sh.clast[tid - 64] = (double)src[sh.cb[tid - 64] + sh.cn[tid - 64] - 1].v;
    const int32_t C = d.C, npairs = d.R * d.C;
    int64_t wp = 0;
    if (tid < npairs) {
        const int r = div_by_c(tid, d.cmag), c = tid - r * C;
        bool live = true;
        if (d.diag)
            live = gram ? (r <= c) : (r < c);
        if (live) {
            const int64_t w = (int64_t)sh.rn[r] + sh.cn[c] - 2;
            wp = (w + kStepBlock - 1) / kStepBlock * kStepBlock;
        }
    }
    // 32-bit work when the tile's step total certainly stays below 2^30
    // (LDS tiles)
    int64_t total;
    LaneSplit<WS> sp;
    const int64_t bound = (int64_t)C * d.rrecs + (int64_t)d.R * d.crecs +
                          (int64_t)kStepBlock * npairs;
    if (bound < ((int64_t)1 << 30)) {
        int32_t t32;
        const int32_t excl =
            block_scan<int32_t>((int32_t)wp, reinterpret_cast<int32_t *>(sh.wsum), &t32);
        pc.sub(0);
        total = t32;
        sp.make_small(t32);
        pc.sub(1);
        if (tid < npairs) {
            sh.pw[tid] = excl;
            // lanes whose first step lies in [excl, excl + wp)
            const int32_t end = excl + (int32_t)wp;
#pragma unroll
            for (int g = 0; g < kGroups; ++g) {
                const int32_t b0 = (int32_t)sp.base[g], b1 = (int32_t)sp.base[g + 1];
                const int32_t per = (int32_t)sp.per[g];
                const int32_t lo = excl > b0 ? excl : b0;
                const int32_t hi = end < b1 ? end : b1;
                if (lo < hi) {
                    for (int32_t j = quot_small(lo - b0 + per - 1, per);
                         b0 + j * per < hi; ++j)
                        sh.pairof[g * kGroupLanes + j] = (int16_t)tid;
                }
            }
        }
    } else {
        const int64_t excl = block_scan<int64_t>(wp, sh.wsum, &total);
        sp.make(total);
        if (tid < npairs) {
            pw64[tid] = excl;
#pragma unroll
            for (int g = 0; g < kGroups; ++g) {
                const int64_t lo = excl > sp.base[g] ? excl : sp.base[g];
                const int64_t hi = excl + wp < sp.base[g + 1] ? excl + wp : sp.base[g + 1];
                if (lo < hi) {
                    for (int64_t j = LaneSplit<WS>::quot(lo - sp.base[g] + sp.per[g] - 1,
                                                        sp.per[g]);
                         sp.base[g] + j * sp.per[g] < hi; ++j)
                        sh.pairof[g * kGroupLanes + j] = (int16_t)tid;
                }
            }
        }
    }
    pc.sub(2);
    if (tid == 0) {
        const bool wide = !(bound < ((int64_t)1 << 30));
        if (wide)
            pw64[npairs] = total;
        else
            sh.pw[npairs] = (int32_t)total;
        sh.pw_wide = wide ? 1 : 0;
        sh.npairs = npairs;
        sh.cmag = d.cmag;
#pragma unroll
        for (int g = 0; g < kGroups; ++g) {
            sh.gper[g] = sp.per[g];
            sh.gbase[g] = sp.base[g];
        }
        sh.gbase[kGroups] = sp.base[kGroups];
    }
    sync_lds();
}

// Persistent tile loop of one workgroup over a ring of three tile
// descriptors in sh.desc (current, next, after next). The queue lane takes
// the ticket of the tile after next before the merge work of the current
// tile and decodes it while the other lanes finish the current tile, so the
// queue's latency stays off the critical path; the next tile (decoded one
// tile earlier) is staged right after finishing. Per tile:
//   scan -> take_next -> merge -> decode_next, finish -> stage_next -> advance
struct TileLoop {
    int cur = 0;
    uint32_t ticket = 0;

    __device__ __forceinline__ int nxt() const { return cur == 2 ? 0 : cur + 1; }
    __device__ __forceinline__ int aft() const { return cur == 0 ? 2 : cur - 1; }

    // decode the first two tiles, stage the first one
    template <typename T, bool Direct, typename Sh>
    __device__ __forceinline__ void start(Sh &sh, const unsigned char *ws,
                                          const int64_t *offsets, Rec<T> *lrec,
                                          const Rec<T> *grec)
    {
        if (threadIdx.x == kQueueLane) {
            tile_decode(sh.desc[0], tile_ticket(ws), ws, offsets);
            tile_decode(sh.desc[1], tile_ticket(ws), ws, offsets);
        }
        sync_lds();
        if (sh.desc[0].tile < hdr_of(ws).ntiles) {
            StageRegs<T, Direct> g;
            stage_load<T, Direct>(g, sh.desc[0], grec, offsets, lrec);
            stage_store<T, Direct>(sh, g, sh.desc[0], lrec);
        }
        sync_lds();
    }
    template <typename Sh>
    __device__ __forceinline__ bool live(const Sh &sh,
                                         const unsigned char *ws) const
    {
        return sh.desc[cur].tile < hdr_of(ws).ntiles;
    }
    // before the merge work of the current tile
    __device__ __forceinline__ void take_next(const unsigned char *ws)
    {
        if (threadIdx.x == kQueueLane)
            ticket = tile_ticket(ws);
    }
    // after the merge work (and its barrier), before finishing
    template <typename Sh>
    __device__ __forceinline__ void decode_next(Sh &sh,
                                                const unsigned char *ws,
                                                const int64_t *offsets)
    {
        if (threadIdx.x == kQueueLane)
            tile_decode(sh.desc[aft()], ticket, ws, offsets);
    }
    // whether there is a next tile (its descriptor, decoded one tile ago)
    template <typename Sh>
    __device__ __forceinline__ bool has_next(const Sh &sh,
                                             const unsigned char *ws) const
    {
        return sh.desc[nxt()].tile < hdr_of(ws).ntiles;
    }
    // staging of the next tile, after finishing the current one; `barrier`
    // when the finishing code reads records or block metadata (otherwise a
    // wave stages as soon as its own finishing work is done)
    template <typename T, bool Direct, typename Sh>
    __device__ __forceinline__ void stage_next(Sh &sh, const unsigned char *ws,
                                               const Rec<T> *grec,
                                               const int64_t *offsets,
                                               Rec<T> *lrec, bool barrier) const
    {
        const TileDesc &n = sh.desc[nxt()];
        if (n.tile >= hdr_of(ws).ntiles)
            return;
        if (barrier)
            sync_lds();
        StageRegs<T, Direct> g;
        stage_load<T, Direct>(g, n, grec, offsets, lrec);
        stage_store<T, Direct>(sh, g, n, lrec);
    }
    __device__ __forceinline__ void advance()
    {
        sync_lds();
        cur = nxt();
    }
};

}  // namespace pcf
