// tile.hpp -- device-side pieces shared by the forward and adjoint tile
// kernels: breakpoint records, the tile queue, LDS staging, the per-pair
// step prefix and the merge-path split (see kernels.hip for the method).
#pragma once

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
// Tile kernel

struct TileShared {
    int64_t pw[kMaxPairs + 1];  // exclusive prefix of padded pair steps
    // partial sums: virtual lane l's share of pair k lands in slot k + l (distinct
    // for all (k, l) because both the pairs and the lanes' step ranges are
    // ordered); each pair then adds its slots in lane order, so the result
    // does not depend on timing
    // (the finished result of pair k goes to slot k + pw[k] / per, also
    // unique per pair, zero-step pairs included)
    double part[kMaxPairs + 2 * kThreads];
    int32_t rn[kMaxBlock], rb[kMaxBlock];  // row PCF rows / record base
    int32_t cn[kMaxBlock], cb[kMaxBlock];  // column PCF rows / record base
    int64_t wsum[kThreads / 64];
    int64_t tile;
    int64_t r_lo, c_lo, rrec0, crec0;
    int64_t obase, ldo, row0, col0;
    int64_t rrecs, crecs;  // records of the row / column block
    int32_t R, C, diag, mirror, global_mode, npairs;
};

constexpr int kSharedHead = (int)((sizeof(TileShared) + 255) / 256 * 256);
static_assert(kSharedHead + kLdsRecordBytes <= 160 * 1024,
              "tile LDS must fit the 160 KiB a gfx950 workgroup can have");

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

// Largest k with pw[k] <= s (the pair holding step s of the tile).
template <typename Shared>
__device__ __forceinline__ int32_t pair_of_step(const Shared &sh, int64_t s)
{
    int32_t lo = 0, hi = sh.npairs - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (sh.pw[mid] <= s)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Pops the next tile from the queue, decodes it, writes the block metadata,
// stages both blocks' records into LDS (unless they do not fit: global
// mode) and prefix-sums the padded step counts of its pairs into sh.pw.
// Diagonal tiles give work to pairs r < c, and to r == c when `gram`.
// Every thread of the workgroup calls it; returns false when the queue is
// empty (uniformly).
template <typename T>
__device__ __forceinline__ bool tile_setup(TileShared &sh, Rec<T> *lrec,
                                           const unsigned char *ws,
                                           const int64_t *offsets, int gram)
{
    const int tid = threadIdx.x;
    const WsHeader &h = hdr_of(ws);
    const int32_t *blocks = reinterpret_cast<const int32_t *>(ws + h.off_blocks);
    const Rec<T> *grec = reinterpret_cast<const Rec<T> *>(ws + h.off_rec);
    uint32_t *counter =
        const_cast<uint32_t *>(reinterpret_cast<const WsHeader *>(ws)->counter);
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
            sh.rrecs = rrecs;
            sh.crecs = crecs;
        }
    }
    __syncthreads();
    if (sh.tile >= h.ntiles)
        return false;
    const int32_t R = sh.R, C = sh.C, npairs = sh.npairs;
    const bool diag = sh.diag != 0, gmode = sh.global_mode != 0;
    const int64_t rrecs = sh.rrecs;

    // block metadata: rows of each PCF and base of its records (LDS index,
    // or global record index in global mode)
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
                                           : rrecs + (roff - sh.crec0)));
    }
    // stage both blocks' records into LDS
    if (!gmode) {
        for (int64_t q = tid; q < rrecs; q += kThreads)
            lrec[q] = grec[sh.rrec0 + q];
        if (!diag)
            for (int64_t q = tid; q < sh.crecs; q += kThreads)
                lrec[rrecs + q] = grec[sh.crec0 + q];
    }
    __syncthreads();

    // padded step count of every pair, prefix-summed
    int64_t wp = 0;
    if (tid < npairs) {
        const int r = tid / C, c = tid - (tid / C) * C;
        bool live = true;
        if (diag)
            live = gram ? (r <= c) : (r < c);
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
    return true;
}

// Even split of a tile's steps over 2 * kThreads virtual lanes (two merge
// chains per lane); a multiple of kStepBlock, at least one block.
__device__ __forceinline__ int64_t steps_per_virtual_lane(int64_t total)
{
    constexpr int kVirtual = 2 * kThreads;
    int64_t per = ((total + kVirtual - 1) / kVirtual + kStepBlock - 1) /
                  kStepBlock * kStepBlock;
    return per < kStepBlock ? kStepBlock : per;
}

}  // namespace pcf
