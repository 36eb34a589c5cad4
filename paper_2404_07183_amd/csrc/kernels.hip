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
#include "tile.hpp"

namespace pcf {

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
    "s_mov_b64 exec, %[sv]"

// Each step first waits until at most two LDS reads are outstanding: the
// two issued by the other chain's step in between (LDS reads complete in
// issue order). The caller ends every block with pcf_lds_drain(), so no
// read is in flight outside a block of steps.
#define PCF_STEP_HEAD "s_waitcnt lgkmcnt(2)\n\t"

__device__ __forceinline__ void pcf_lds_drain()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

#define PCF_RECBITS_f64 "128"
#define PCF_RECBITS_f32 "64"

template <typename T, int HK> struct AsmStep;

// Head of a step for a chain that runs alone (no other chain's reads in
// flight): wait for all outstanding LDS reads.
#define PCF_STEP_HEAD_SOLO "s_waitcnt lgkmcnt(0)\n\t"

#define PCF_ASM_OPERANDS                                                      \
    : [ra] "+v"(ra), [rb] "+v"(rb), [ia] "+v"(ia), [ib] "+v"(ib),           \
      [acc] "+v"(acc), [y] "=&v"(y), [d] "=&v"(d), [dv] "=&v"(dv),          \
      [sv] "=&s"(sv)                                                        \
    : [nf] "v"(ra.x), [ng] "v"(rb.x), [a] "v"(ra.y), [b] "v"(rb.y),         \
      [x] "v"(x)                                                            \
    : "vcc", "scc", "memory"

template <> struct AsmStep<double, kAbs> {
    template <bool SOLO>
    __device__ __forceinline__ static void run(d2v &ra, d2v &rb, uint32_t &ia,
                                               uint32_t &ib, double x, double &y,
                                               double &acc)
    {
        double d, dv;
        uint64_t sv;
        if constexpr (SOLO)
            asm volatile(PCF_STEP_HEAD_SOLO "v_min_f64 %[y], %[nf], %[ng]\n\t"
                     "v_add_f64 %[d], %[y], -%[x]\n\t"
                     "v_add_f64 %[dv], %[a], -%[b]\n\t"
                     "v_fma_f64 %[acc], |%[dv]|, %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f64, "16")
                     PCF_ASM_OPERANDS);
        else
            asm volatile(PCF_STEP_HEAD "v_min_f64 %[y], %[nf], %[ng]\n\t"
                     "v_add_f64 %[d], %[y], -%[x]\n\t"
                     "v_add_f64 %[dv], %[a], -%[b]\n\t"
                     "v_fma_f64 %[acc], |%[dv]|, %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f64, "16")
                     PCF_ASM_OPERANDS);
    }
};
template <> struct AsmStep<double, kSqr> {
    template <bool SOLO>
    __device__ __forceinline__ static void run(d2v &ra, d2v &rb, uint32_t &ia,
                                               uint32_t &ib, double x, double &y,
                                               double &acc)
    {
        double d, dv;
        uint64_t sv;
        if constexpr (SOLO)
            asm volatile(PCF_STEP_HEAD_SOLO "v_min_f64 %[y], %[nf], %[ng]\n\t"
                     "v_add_f64 %[d], %[y], -%[x]\n\t"
                     "v_add_f64 %[dv], %[a], -%[b]\n\t"
                     "v_mul_f64 %[d], %[dv], %[d]\n\t"
                     "v_fma_f64 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f64, "16")
                     PCF_ASM_OPERANDS);
        else
            asm volatile(PCF_STEP_HEAD "v_min_f64 %[y], %[nf], %[ng]\n\t"
                     "v_add_f64 %[d], %[y], -%[x]\n\t"
                     "v_add_f64 %[dv], %[a], -%[b]\n\t"
                     "v_mul_f64 %[d], %[dv], %[d]\n\t"
                     "v_fma_f64 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f64, "16")
                     PCF_ASM_OPERANDS);
    }
};
template <> struct AsmStep<double, kProd> {
    template <bool SOLO>
    __device__ __forceinline__ static void run(d2v &ra, d2v &rb, uint32_t &ia,
                                               uint32_t &ib, double x, double &y,
                                               double &acc)
    {
        double d, dv;
        uint64_t sv;
        if constexpr (SOLO)
            asm volatile(PCF_STEP_HEAD_SOLO "v_min_f64 %[y], %[nf], %[ng]\n\t"
                     "v_add_f64 %[d], %[y], -%[x]\n\t"
                     "v_mul_f64 %[dv], %[a], %[b]\n\t"
                     "v_fma_f64 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f64, "16")
                     PCF_ASM_OPERANDS);
        else
            asm volatile(PCF_STEP_HEAD "v_min_f64 %[y], %[nf], %[ng]\n\t"
                     "v_add_f64 %[d], %[y], -%[x]\n\t"
                     "v_mul_f64 %[dv], %[a], %[b]\n\t"
                     "v_fma_f64 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f64, "16")
                     PCF_ASM_OPERANDS);
    }
};
template <> struct AsmStep<float, kAbs> {
    template <bool SOLO>
    __device__ __forceinline__ static void run(f2v &ra, f2v &rb, uint32_t &ia,
                                               uint32_t &ib, float x, float &y,
                                               float &acc)
    {
        float d, dv;
        uint64_t sv;
        if constexpr (SOLO)
            asm volatile(PCF_STEP_HEAD_SOLO "v_min_f32 %[y], %[nf], %[ng]\n\t"
                     "v_sub_f32 %[d], %[y], %[x]\n\t"
                     "v_sub_f32 %[dv], %[a], %[b]\n\t"
                     "v_fma_f32 %[acc], |%[dv]|, %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f32, "8")
                     PCF_ASM_OPERANDS);
        else
            asm volatile(PCF_STEP_HEAD "v_min_f32 %[y], %[nf], %[ng]\n\t"
                     "v_sub_f32 %[d], %[y], %[x]\n\t"
                     "v_sub_f32 %[dv], %[a], %[b]\n\t"
                     "v_fma_f32 %[acc], |%[dv]|, %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f32, "8")
                     PCF_ASM_OPERANDS);
    }
};
template <> struct AsmStep<float, kSqr> {
    template <bool SOLO>
    __device__ __forceinline__ static void run(f2v &ra, f2v &rb, uint32_t &ia,
                                               uint32_t &ib, float x, float &y,
                                               float &acc)
    {
        float d, dv;
        uint64_t sv;
        if constexpr (SOLO)
            asm volatile(PCF_STEP_HEAD_SOLO "v_min_f32 %[y], %[nf], %[ng]\n\t"
                     "v_sub_f32 %[d], %[y], %[x]\n\t"
                     "v_sub_f32 %[dv], %[a], %[b]\n\t"
                     "v_mul_f32 %[d], %[dv], %[d]\n\t"
                     "v_fma_f32 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f32, "8")
                     PCF_ASM_OPERANDS);
        else
            asm volatile(PCF_STEP_HEAD "v_min_f32 %[y], %[nf], %[ng]\n\t"
                     "v_sub_f32 %[d], %[y], %[x]\n\t"
                     "v_sub_f32 %[dv], %[a], %[b]\n\t"
                     "v_mul_f32 %[d], %[dv], %[d]\n\t"
                     "v_fma_f32 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f32, "8")
                     PCF_ASM_OPERANDS);
    }
};
template <> struct AsmStep<float, kProd> {
    template <bool SOLO>
    __device__ __forceinline__ static void run(f2v &ra, f2v &rb, uint32_t &ia,
                                               uint32_t &ib, float x, float &y,
                                               float &acc)
    {
        float d, dv;
        uint64_t sv;
        if constexpr (SOLO)
            asm volatile(PCF_STEP_HEAD_SOLO "v_min_f32 %[y], %[nf], %[ng]\n\t"
                     "v_sub_f32 %[d], %[y], %[x]\n\t"
                     "v_mul_f32 %[dv], %[a], %[b]\n\t"
                     "v_fma_f32 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f32, "8")
                     PCF_ASM_OPERANDS);
        else
            asm volatile(PCF_STEP_HEAD "v_min_f32 %[y], %[nf], %[ng]\n\t"
                     "v_sub_f32 %[d], %[y], %[x]\n\t"
                     "v_mul_f32 %[dv], %[a], %[b]\n\t"
                     "v_fma_f32 %[acc], %[dv], %[d], %[acc]\n\t"
                     PCF_STEP_TAIL(f32, "8")
                     PCF_ASM_OPERANDS);
    }
};

// One merge chain: a contiguous run of the tile's steps, possibly over
// several pairs. Its partial sum of pair k goes to sh.part[k + vl].
template <typename T>
struct Chain {
    typename RecVec<T>::type ra, rb;  // current (end time, value) records
    uint32_t ia, ib;                  // their LDS byte addresses
    T x0, x1;                         // start of the current cell (alternating)
    double acc;
    int64_t left;                     // steps left in pair k
    int32_t k, vl;
};

template <typename T, typename Shared>
__device__ __forceinline__ void chain_begin(Chain<T> &ch, Shared &sh,
                                            const Rec<T> *lrec, int64_t s,
                                            int32_t vl, int32_t C)
{
    typedef typename RecVec<T>::type V;
    const V *lv = reinterpret_cast<const V *>(lrec);
    const int32_t k = pair_of_step(sh, s);
    const int64_t d = s - sh.pw[k];
    const int r = k / C, c = k - (k / C) * C;
    int32_t i0, j0;
    T x;
    pair_start<T>(lrec, sh.rb[r], sh.rn[r], sh.cb[c], sh.cn[c], d, i0, j0, x);
    ch.ra = lv[i0];
    ch.rb = lv[j0];
    ch.ia = lds_address(&lrec[i0]);
    ch.ib = lds_address(&lrec[j0]);
    ch.x0 = x;
    ch.acc = 0.0;
    ch.left = sh.pw[k + 1] - sh.pw[k] - d;
    ch.k = k;
    ch.vl = vl;
}

// Between blocks: a chain that finished its pair records it and moves to
// the next pair with steps (a rare, divergent branch).
template <typename T, typename Shared>
__device__ __forceinline__ void chain_advance(Chain<T> &ch, Shared &sh,
                                              const Rec<T> *lrec, int32_t C)
{
    if (ch.left != 0)
        return;
    typedef typename RecVec<T>::type V;
    const V *lv = reinterpret_cast<const V *>(lrec);
    sh.part[ch.k + ch.vl] = ch.acc;
    ch.acc = 0.0;
    int32_t k = ch.k + 1;
    while (k < sh.npairs && sh.pw[k + 1] == sh.pw[k])
        ++k;
    ch.k = k;
    ch.left = sh.pw[k + 1] - sh.pw[k];
    const int r = k / C, c = k - (k / C) * C;
    const int32_t A = sh.rb[r], B = sh.cb[c];
    ch.ra = lv[A];
    ch.rb = lv[B];
    ch.ia = lds_address(&lrec[A]);
    ch.ib = lds_address(&lrec[B]);
    ch.x0 = T(0);
}

// Two chains of one lane, steps interleaved so that each chain's record
// reads are in flight while the other chain computes.
template <typename T, int HK>
__device__ __forceinline__ void block_pair(Chain<T> &c0, Chain<T> &c1)
{
    T p0 = T(0), p1 = T(0);
#pragma unroll
    for (int u = 0; u < kStepBlock; u += 2) {
        AsmStep<T, HK>::template run<false>(c0.ra, c0.rb, c0.ia, c0.ib, c0.x0, c0.x1, p0);
        AsmStep<T, HK>::template run<false>(c1.ra, c1.rb, c1.ia, c1.ib, c1.x0, c1.x1, p1);
        AsmStep<T, HK>::template run<false>(c0.ra, c0.rb, c0.ia, c0.ib, c0.x1, c0.x0, p0);
        AsmStep<T, HK>::template run<false>(c1.ra, c1.rb, c1.ia, c1.ib, c1.x1, c1.x0, p1);
    }
    pcf_lds_drain();
    c0.acc += (double)p0;
    c1.acc += (double)p1;
    c0.left -= kStepBlock;
    c1.left -= kStepBlock;
}

template <typename T, int HK>
__device__ __forceinline__ void block_solo(Chain<T> &c0)
{
    T p0 = T(0);
#pragma unroll
    for (int u = 0; u < kStepBlock; u += 2) {
        AsmStep<T, HK>::template run<true>(c0.ra, c0.rb, c0.ia, c0.ib, c0.x0, c0.x1, p0);
        AsmStep<T, HK>::template run<true>(c0.ra, c0.rb, c0.ia, c0.ib, c0.x1, c0.x0, p0);
    }
    pcf_lds_drain();
    c0.acc += (double)p0;
    c0.left -= kStepBlock;
}

// This lane's two chains: virtual lanes 2*lane and 2*lane+1 of the tile's
// even split, steps [s0, e0) and [s1, e1) with e0 == s1 (e1 - s1 <= e0 - s0,
// only the tile's last lanes are short). Both run in one block loop.
template <typename T, int HK, typename Shared>
__device__ __forceinline__ void lane_chains_lds(Shared &sh, const Rec<T> *lrec,
                                                int64_t s0, int64_t e0,
                                                int64_t s1, int64_t e1,
                                                int32_t lane, int32_t C)
{
    const int64_t nb0 = (e0 - s0) / kStepBlock;
    const int64_t nb1 = (e1 > s1) ? (e1 - s1) / kStepBlock : 0;
    Chain<T> c0, c1;
    chain_begin(c0, sh, lrec, s0, 2 * lane, C);
    if (nb1 > 0)
        chain_begin(c1, sh, lrec, s1, 2 * lane + 1, C);
    int64_t blk = 0;
    for (; blk < nb1; ++blk) {
        chain_advance(c0, sh, lrec, C);
        chain_advance(c1, sh, lrec, C);
        block_pair<T, HK>(c0, c1);
    }
    for (; blk < nb0; ++blk) {
        chain_advance(c0, sh, lrec, C);
        block_solo<T, HK>(c0);
    }
    sh.part[c0.k + c0.vl] = c0.acc;
    if (nb1 > 0)
        sh.part[c1.k + c1.vl] = c1.acc;
}

// Single-chain C++ loop (h = |a-b|^p, whose step is not hand-written).
template <typename T, int HK, typename Shared>
__device__ __forceinline__ void chain_cpp(Shared &sh, const Rec<T> *lrec,
                                          int64_t s, int64_t e, int32_t vl,
                                          int32_t C, T p)
{
    int32_t k = pair_of_step(sh, s);
    int64_t d = s - sh.pw[k];
    int64_t left = sh.pw[k + 1] - sh.pw[k] - d;
    int32_t ia, ib;
    T x;
    {
        const int r = k / C, c = k - (k / C) * C;
        pair_start<T>(lrec, sh.rb[r], sh.rn[r], sh.cb[c], sh.cn[c], d, ia, ib, x);
    }
    Rec<T> ra = lrec[ia], rb = lrec[ib];
    double acc = 0.0;
    const int64_t nblk = (e - s) / kStepBlock;
    for (int64_t blk = 0; blk < nblk; ++blk) {
        if (left == 0) {
            sh.part[k + vl] = acc;
            acc = 0.0;
            ++k;
            while (k < sh.npairs && sh.pw[k + 1] == sh.pw[k])
                ++k;
            left = sh.pw[k + 1] - sh.pw[k];
            const int r = k / C, c = k - (k / C) * C;
            ia = sh.rb[r];
            ib = sh.cb[c];
            ra = lrec[ia];
            rb = lrec[ib];
            x = T(0);
        }
        T part = T(0);
#pragma unroll
        for (int u = 0; u < kStepBlock; ++u) {
            const T y = ra.t <= rb.t ? ra.t : rb.t;
            part = fma(hval<T, HK>(ra.v, rb.v, p), y - x, part);
            x = y;
            if (ra.t <= rb.t)
                ra = lrec[++ia];
            else
                rb = lrec[++ib];
        }
        acc += (double)part;
        left -= kStepBlock;
    }
    sh.part[k + vl] = acc;
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
    const Rec<T> *grec = reinterpret_cast<const Rec<T> *>(ws + h.off_rec);
    const int64_t *offsets = args.offsets;
    const T p = (T)args.p;

    for (;;) {
        if (!tile_setup<T>(sh, lrec, ws, offsets, args.gram))
            break;
        const int32_t R = sh.R, C = sh.C, npairs = sh.npairs;
        const bool diag = sh.diag != 0, gmode = sh.global_mode != 0;
        const int64_t total = sh.pw[npairs];

        // the tile's steps split evenly over 2 * kThreads virtual lanes, two
        // per lane (see lane_chains_lds)
        const int64_t per = steps_per_virtual_lane(total);
        const int64_t s0 = (int64_t)(2 * tid) * per;
        const int64_t e0 = (s0 + per < total) ? s0 + per : total;
        const int64_t s1 = e0;
        const int64_t e1 = (s1 + per < total) ? s1 + per : total;
        if (s0 < e0) {
            if (gmode) {
                for (int q = 0; q < 2; ++q) {
                    int64_t s = q ? s1 : s0;
                    const int64_t e = q ? e1 : e0;
                    if (s >= e)
                        continue;
                    int32_t k = pair_of_step(sh, s);
                    int64_t d = s - sh.pw[k];
                    while (s < e) {
                        const int r = k / C, c = k - (k / C) * C;
                        const int64_t len = sh.pw[k + 1] - sh.pw[k];
                        const int64_t m = (len - d < e - s) ? len - d : e - s;
                        sh.part[k + 2 * tid + q] = run_pair_global<T, HK>(
                            grec, sh.rb[r], sh.rn[r], sh.cb[c], sh.cn[c], d, m, p);
                        s += m;
                        d = 0;
                        ++k;
                        while (k < npairs && sh.pw[k + 1] == sh.pw[k])
                            ++k;
                    }
                }
            } else if constexpr (HK == kPow) {
                chain_cpp<T, HK>(sh, lrec, s0, e0, 2 * tid, C, p);
                if (s1 < e1)
                    chain_cpp<T, HK>(sh, lrec, s1, e1, 2 * tid + 1, C, p);
            } else {
                lane_chains_lds<T, HK>(sh, lrec, s0, e0, s1, e1, tid, C);
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
            sh.part[k + b0 / per] = val;
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
                const int kk = r * C + c;
                const double val = sh.part[kk + sh.pw[kk] / per];
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
