// kernels.hip -- gfx950 kernels for pairwise integrated combinations of PCFs.
//
// Method (paper, Section 3, Algorithms "IterateRectangles" and
// "CombineIntegrate"): for a pair (f, g) walk both sorted breakpoint lists
// once, left to right; every step closes one cell [x, y) of the common
// refinement with y the earlier of the two next breakpoints, adds
// h(f(x), g(x)) * (y - x) and moves the pointer(s) whose next breakpoint is
// y. The paper's pair loop is used as is; what is specific to this library:
//
//  * Breakpoint records. Row k of a PCF is packed as (t_{k+1}, v_k): the
//    value of piece k and the time where it ends; the last piece ends at a
//    finite sentinel S (largest finite value of the type), followed by
//    kPad copies of (S, v_last). A step then needs one record load, of the
//    side that advances.
//  * Ties. On equal next times only one side advances; the other advances
//    in the following step, whose cell has width 0 and adds exactly 0.
//    Every pair therefore takes exactly (n_f - 1) + (n_g - 1) steps (padded
//    to a multiple of kStepBlock with sentinel steps that add 0) -- known
//    before the loop, so work can be split exactly. The merge-path split
//    lets the row side go first; the loop lets the piece loaded last go
//    first. Both orders give the same cells of positive width, and a lane's
//    share starts after a whole number of merged breakpoints, whose last
//    time does not depend on the order, so the shares fit together.
//  * Tiles and LDS. A workgroup takes a tile (row block x column block) from
//    a persistent queue, copies both blocks' records into LDS and splits the
//    tile's total step count over its 1024 lanes, one contiguous run of
//    steps per lane, longer runs for the waves the SIMDs issue first (see
//    LaneSplit). A run may start inside a pair: its starting
//    pointers come from a merge-path binary search on the pair's diagonal,
//    and partial sums of one pair meet in LDS slots, added in lane order
//    (deterministic). No lane waits for a longer pair, whatever the length
//    mix.
//  * The step (see Chain): one full-wave LDS read per step, no divergence.
//  * Output. Results are finished (root, unbounded-tail rule) in LDS and
//    written row by row, then transposed, both coalesced.
#include <hip/hip_runtime.h>

#include <float.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <set>
#include <utility>

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
// Grid-stride over rows; P comes from offsets[n] on the device. The set's
// records start at record rec_base (0, or past a first set's records when
// two sets share one record array).
template <typename T>
__global__ void pack_records(const int64_t *__restrict__ offsets, int64_t n,
                             const T *__restrict__ t, const T *__restrict__ v,
                             unsigned char *ws, int64_t rec_base)
{
    const WsHeader &h = hdr_of(ws);
    Rec<T> *rec = reinterpret_cast<Rec<T> *>(ws + h.off_rec) + rec_base;
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
// The merge chain.
//
// h is symmetric in its two arguments, so a chain does not track which PCF
// a piece belongs to: P holds the piece loaded last, Q the other one, each
// as (end time, value) plus a pointer to its record. One step closes the
// cell [x, y), y = min(P.t, Q.t); the piece that ends there (P on equal
// times) is replaced by its successor, which is always loaded into P (the
// piece that goes on becomes Q). Every lane of a wave loads one record per
// step: one full-wave LDS read, no divergent branch. The end time of the
// piece that goes on is max(P.t, Q.t), which saves two selects.

template <typename T> struct GlobalWalk {
    typedef typename RecVec<T>::type V;
    const V *pP, *pQ;

    __device__ __forceinline__ void set(const Rec<T> *base, int32_t iP, int32_t iQ)
    {
        pP = reinterpret_cast<const V *>(base + iP);
        pQ = reinterpret_cast<const V *>(base + iQ);
    }
    __device__ __forceinline__ static V at(const Rec<T> *base, int32_t i)
    {
        return *reinterpret_cast<const V *>(base + i);
    }
    template <int K>
    __device__ __forceinline__ V advance(bool p_ends)
    {
        const V *n = p_ends ? pP : pQ;
        pQ = p_ends ? pQ : pP;
        pP = n + 1;
        return *pP;
    }
    __device__ __forceinline__ void end_block() {}
};

template <typename T, typename Walk>
struct Chain {
    typename RecVec<T>::type P;  // piece loaded last: (end time, value)
    T tQ, vQ;                    // the other piece
    Walk w;                      // record addresses
    T x;          // start of the current cell
    double acc;   // sum over the current pair (FP64 for both types)
    int32_t left; // steps left in the current pair (rows < 2^30 per PCF)
    int32_t k, r, c;         // current pair: index r * C + c, row, column
    int32_t rb, rn, cb, cn;  // record base and rows of its two PCFs

    __device__ __forceinline__ void load(const Rec<T> *base, int32_t iP, int32_t iQ)
    {
        w.set(base, iP, iQ);
        P = Walk::at(base, iP);
        const typename RecVec<T>::type Q = Walk::at(base, iQ);
        tQ = Q.x;
        vQ = Q.y;
    }
};

template <int K, typename T, int HK, typename Walk>
__device__ __forceinline__ void chain_step(Chain<T, Walk> &ch, T &part, T p)
{
    const T tP = ch.P.x, tQ = ch.tQ;
    const T y = min_raw(tP, tQ);
    part = fma(hval<T, HK>(ch.P.y, ch.vQ, p), y - ch.x, part);
    ch.x = y;
    const bool c = tP <= tQ;
    ch.vQ = c ? ch.vQ : ch.P.y;
    ch.tQ = max_raw(tP, tQ);
    ch.P = ch.w.template advance<K>(c);
}

template <typename T, int HK, typename Walk, int... Ks>
__device__ __forceinline__ void chain_block(Chain<T, Walk> &ch, T &part, T p,
                                            std::integer_sequence<int, Ks...>)
{
    (chain_step<Ks, T, HK>(ch, part, p), ...);
    ch.w.end_block();
}

// Padded merge steps of a pair of PCFs with na and nb rows (as in the scan;
// below 2^31 since the planner admits fewer than 2^30 rows per PCF).
__device__ __forceinline__ int32_t pair_steps(int32_t na, int32_t nb)
{
    return (na + nb - 2 + kStepBlock - 1) & ~(kStepBlock - 1);
}

// Starting state at step d of pair k (merge-path split).
template <typename T, typename Walk, typename Shared>
__device__ __forceinline__ void chain_begin(Chain<T, Walk> &ch, const Shared &sh,
                                            const Rec<T> *base, int32_t k,
                                            int64_t d, int32_t C)
{
    const int r = div_by_c(k, sh.cmag), c = k - r * C;
    ch.k = k;
    ch.r = r;
    ch.c = c;
    ch.rb = sh.rb[r];
    ch.rn = sh.rn[r];
    ch.cb = sh.cb[c];
    ch.cn = sh.cn[c];
    int32_t i0, j0;
    T x;
    pair_start<T>(base, ch.rb, ch.rn, ch.cb, ch.cn, d, i0, j0, x);
    ch.load(base, i0, j0);
    ch.x = x;
    ch.acc = 0.0;
    ch.left = pair_steps(ch.rn, ch.cn) - (int32_t)d;
}

// Moves a chain that finished its pair to the next pair with steps, in the
// tile's row-major pair order. Blocks of consecutive PCFs are contiguous in
// the record arrays, so the next PCF's records start right after this one's
// padding. In the common case (next column, same row) the new pair's first
// two records are read together with the new column's row count (one LDS
// round trip); a row change reads the new row's metadata first. On diagonal
// tiles a row's live pairs start at column r + 1 (r with `gram`). A pair
// without steps (two one-row PCFs) is skipped; the caller has steps left,
// so a next pair with steps exists.
template <typename T, typename Walk, typename Shared>
__device__ __forceinline__ void chain_next_pair(Chain<T, Walk> &ch, const Shared &sh,
                                                const Rec<T> *base, int32_t C,
                                                bool diag, int gram)
{
    int32_t k = ch.k + 1, r = ch.r, c = ch.c + 1, rb = ch.rb, rn = ch.rn;
    int32_t cb = ch.cb + ch.cn + kPad;
    if (c >= C) {
        // next row (k was (r - 1) * C + C = r * C)
        rb += rn + kPad;
        ++r;
        rn = sh.rn[r];
        c = diag ? (gram ? r : r + 1) : 0;
        k += c;
        cb = sh.cb[c];
    }
    // the new column's row count and the pair's first records, together
    int32_t cn = sh.cn[c];
    ch.load(base, rb, cb);
    while (pair_steps(rn, cn) == 0) {
        // a pair without steps (two one-row PCFs): skip it (rare)
        ++k;
        ++c;
        cb += cn + kPad;
        if (c >= C) {
            rb += rn + kPad;
            ++r;
            rn = sh.rn[r];
            c = diag ? (gram ? r : r + 1) : 0;
            k += c;
            cb = sh.cb[c];
        }
        cn = sh.cn[c];
        ch.load(base, rb, cb);
    }
    ch.k = k;
    ch.r = r;
    ch.c = c;
    ch.rb = rb;
    ch.rn = rn;
    ch.cb = cb;
    ch.cn = cn;
    ch.x = T(0);
    ch.acc = 0.0;
    ch.left = pair_steps(rn, cn);
}

// This lane's share of the tile: nblk blocks of kStepBlock steps (pair
// boundaries fall between blocks), starting at step d0 of pair k; its
// partial sum of pair k' goes to sh.part[k' + vl].
template <typename T, int HK, typename Walk, typename Shared>
__device__ __forceinline__ void lane_chain(Shared &sh, const Rec<T> *base,
                                           int64_t d0, int32_t nblk, int32_t k,
                                           int32_t vl, int32_t C, bool diag,
                                           int gram, T p, PhaseClock &pc)
{
    Chain<T, Walk> ch;
    chain_begin(ch, sh, base, k, d0, C);
    pc.mark(kPhaseStart);
    for (int32_t blk = nblk; blk > 0; --blk) {
        const unsigned long long t0 = pc.now();
        const bool sw = __builtin_amdgcn_ballot_w64(ch.left == 0) != 0;
        if (ch.left == 0) {
            // next pair (a rare, divergent branch)
            sh.part[ch.k + vl] = ch.acc;
            chain_next_pair(ch, sh, base, C, diag, gram);
        }
        pc.sw_add(t0, sw);
        T part = T(0);
        chain_block<T, HK>(ch, part, p, std::make_integer_sequence<int, kStepBlock>());
        ch.acc += (double)part;
        ch.left -= kStepBlock;
    }
    sh.part[ch.k + vl] = ch.acc;
}

template <typename T, int HK, int RT>
__global__ __launch_bounds__(kThreads) void pairwise_tiles(FwdArgs args)
{
    extern __shared__ __align__(16) unsigned char smem[];
    TileShared &sh = *reinterpret_cast<TileShared *>(smem);
    Rec<T> *lrec = reinterpret_cast<Rec<T> *>(smem + kSharedHead);
    int64_t *pw64 = reinterpret_cast<int64_t *>(lrec);  // wide step prefix
    const int tid = threadIdx.x;
    const unsigned char *ws = args.ws;
    const WsHeader &h = hdr_of(ws);
    const Rec<T> *grec = reinterpret_cast<const Rec<T> *>(ws + h.off_rec);
    const int64_t *offsets = args.offsets;
    const T p = (T)args.p;
    T *out = reinterpret_cast<T *>(args.out);

    PhaseClock pc;
    TileLoop loop;
    loop.start<T, false>(sh, ws, offsets, lrec, grec);
    pc.mark(-1);
    while (loop.live(sh, ws)) {
        const TileDesc &D = sh.desc[loop.cur];
        const bool gmode = D.global_mode != 0;
        tile_scan<T>(sh, D, args.gram, gmode ? grec : lrec, pw64, pc);
        const int32_t C = D.C, npairs = sh.npairs;
        const bool diag = D.diag != 0;
        const int64_t total = pw_at(sh, pw64, npairs);
        const int32_t run = tid;  // the run of steps this lane executes
        pc.mark(kPhaseScan);
        pc.tile(total);

        loop.take_next(ws);
        // this lane's share of the tile's steps
        int64_t s0, e0;
        lane_steps(sh, run, total, s0, e0);
        const int32_t k0 = s0 < e0 ? sh.pairof[run] : 0;
        if (s0 < e0) {
            const int64_t d0 = s0 - pw_at(sh, pw64, k0);
            const int32_t nblk = (int32_t)((e0 - s0) / kStepBlock);
            if (gmode)
                lane_chain<T, HK, GlobalWalk<T>>(sh, grec, d0, nblk, k0, run, C,
                                                 diag, args.gram, p, pc);
            else
                lane_chain<T, HK, LdsWalk<T>>(sh, lrec, d0, nblk, k0, run, C,
                                              diag, args.gram, p, pc);
        } else {
            pc.mark(kPhaseStart);
        }
        pc.mark(kPhaseMerge);
        // the next tile's staging loads, issued as soon as this wave's merge
        // work is done (they only fill registers; the records are stored to
        // LDS after the barrier and the finishing reads)
        const bool has_next = loop.has_next(sh, ws);
        StageRegs<T, false> next;
        if (has_next)
            stage_load<T, false>(next, sh.desc[loop.nxt()], grec, offsets, lrec);
        sync_lds();
        pc.mark(kPhaseMergeWait);
        loop.decode_next(sh, ws, offsets);
        pc.mark(kPhaseStageIssue);

        // finish: unbounded-tail rule, root. A tile has at most kThreads
        // pairs, so a thread finishes at most one; its results are stored
        // after the staging below, so that the staging's wait for its loads
        // does not also wait for these stores.
        static_assert(kMaxPairs <= kThreads, "one pair per thread when finishing");
        bool wr = false, wr_mirror = false;
        T res = T(0);
        int64_t at0 = 0, at1 = 0;
        if (tid < npairs) {
            const int k = tid;
            const int r = div_by_c(k, D.cmag), c = k - r * C;
            if (!(diag && r > c)) {
                // the lanes holding the pair's first and last steps (none for
                // a pair without steps)
                const int64_t b0 = pw_at(sh, pw64, k), b1 = pw_at(sh, pw64, k + 1);
                int32_t l = 0, l1 = -1;
                if (b1 > b0) {
                    l = lane_of(sh, b0);
                    l1 = lane_of(sh, b1 - 1);
                }
                const T lr = (T)sh.rlast[r], lc = (T)sh.clast[c];
                // the pair's partial sums in lane order, loads batched
                double val = 0.0;
                for (; l + 3 <= l1; l += 4) {
                    const double q0 = sh.part[k + l], q1 = sh.part[k + l + 1];
                    const double q2 = sh.part[k + l + 2], q3 = sh.part[k + l + 3];
                    val = (((val + q0) + q1) + q2) + q3;
                }
                for (; l <= l1; ++l)
                    val += sh.part[k + l];
                const T ht = hval<T, HK>(lr, lc, p);
                if (ht != T(0))
                    val = ht > T(0) ? INFINITY : -INFINITY;
                if constexpr (RT == kRootSqrt)
                    val = sqrt(val);
                else if constexpr (RT == kRootPow)
                    val = pow(val, args.inv_p);
                const int64_t i = D.r_lo + r, j = D.c_lo + c;
                if (args.accumulate != 0)  // a term of a sum (no root: checked on the host)
                    val *= args.coef;
                res = (T)val;
                wr = true;
                at0 = D.obase + (i - D.row0) * D.ldo + (j - D.col0);
                wr_mirror = D.mirror && !(diag && r == c);
                at1 = D.obase + (j - D.row0) * D.ldo + (i - D.col0);
            }
        }
        pc.mark(kPhaseFinish);
        if (has_next)
            stage_store<T, false>(sh, next, sh.desc[loop.nxt()], lrec);
        pc.mark(kPhaseStageStore);
        // (i, j) and, mirrored, (j, i); nothing waits for these stores until
        // the next tile's staging
        if (wr) {
            if (args.accumulate == 1) {
                // each entry has one writer per launch; the terms' launches
                // are ordered on the stream
                out[at0] += res;
                if (wr_mirror)
                    out[at1] += res;
            } else {
                out[at0] = res;
                if (wr_mirror)
                    out[at1] = res;
            }
        }
        loop.advance();
        pc.mark(kPhaseAdvance);
    }
    pc.flush((tid & 63) == 0 ? tid >> 6 : -1);
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the C-ABI layer).

size_t tile_shared_bytes(int rec_bytes, bool backward)
{
    // the forward kernel keeps its tile state at the start of the dynamic
    // LDS, the adjoint in static LDS (with two 64-bit gradient slots per
    // record after its records)
    if (backward)
        return (size_t)adj_lds_records(rec_bytes) * (rec_bytes + 16);
    return (size_t)kSharedHead + (size_t)(kLdsRecordBytes / rec_bytes) * rec_bytes;
}

template <typename T>
hipError_t launch_pack(const int64_t *offsets, int64_t n, const void *t,
                       const void *v, unsigned char *ws, int64_t P,
                       hipStream_t s, int64_t rec_base)
{
    if (P <= 0)
        return hipSuccess;
    int64_t blocks = (P + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(pack_records<T>, dim3((unsigned)blocks), dim3(256), 0, s,
                       offsets, n, (const T *)t, (const T *)v, ws, rec_base);
    return hipGetLastError();
}

// The offsets of set X followed by those of set Y shifted by X's row count:
// one CSR over both sets (device; Y's rows come after X's).
__global__ void concat_offsets(const int64_t *__restrict__ xo, int64_t nx,
                               const int64_t *__restrict__ yo, int64_t ny,
                               int64_t *__restrict__ out)
{
    const int64_t px = xo[nx];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= nx + ny;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = i <= nx ? xo[i] : px + yo[i - nx];
}

hipError_t launch_concat_offsets(const int64_t *xo, int64_t nx, const int64_t *yo,
                                 int64_t ny, int64_t *out, hipStream_t s)
{
    int64_t blocks = (nx + ny + 1 + 255) / 256;
    if (blocks > 1024)
        blocks = 1024;
    hipLaunchKernelGGL(concat_offsets, dim3((unsigned)blocks), dim3(256), 0, s, xo,
                       nx, yo, ny, out);
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

hipError_t ensure_dynamic_lds(const void *kernel, int bytes)
{
    static std::mutex mu;
    static std::set<std::pair<const void *, int>> done;  // (kernel, device)
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lock(mu);
    if (done.count({kernel, dev}))
        return hipSuccess;
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        done.insert({kernel, dev});
    return e;
}

hipError_t launch_reset(unsigned char *ws, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, ws);
    return hipGetLastError();
}

template <typename T, int HK, int RT>
static hipError_t launch_fwd_t(const FwdArgs &a, int grid, hipStream_t s)
{
    const size_t shm = tile_shared_bytes((int)sizeof(Rec<T>), false);
    const hipError_t e = ensure_dynamic_lds(
        reinterpret_cast<const void *>(&pairwise_tiles<T, HK, RT>), (int)shm);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((pairwise_tiles<T, HK, RT>), dim3(grid), dim3(kThreads),
                       shm, s, a);
    return hipGetLastError();
}

// The (h, root) combinations the entry points use: |a-b| and ab without a
// root, (a-b)^2 with or without sqrt, |a-b|^p with or without the p-th root
// (integer p: squaring; p = k + 1/2: squaring and one sqrt; any other p:
// 2^(p log2 |a-b|)).
template <typename T>
static hipError_t launch_fwd_dtype(int hk, const FwdArgs &a, int grid,
                                   hipStream_t s)
{
    switch (hk) {
    case kAbs: return launch_fwd_t<T, kAbs, kRootNone>(a, grid, s);
    case kProd: return launch_fwd_t<T, kProd, kRootNone>(a, grid, s);
    case kSqr:
        return a.root == kRootSqrt ? launch_fwd_t<T, kSqr, kRootSqrt>(a, grid, s)
                                   : launch_fwd_t<T, kSqr, kRootNone>(a, grid, s);
    case kPowHalf:
        return a.root == kRootPow ? launch_fwd_t<T, kPowHalf, kRootPow>(a, grid, s)
                                  : launch_fwd_t<T, kPowHalf, kRootNone>(a, grid, s);
    case kPowInt:
        return a.root == kRootPow ? launch_fwd_t<T, kPowInt, kRootPow>(a, grid, s)
                                  : launch_fwd_t<T, kPowInt, kRootNone>(a, grid, s);
    default:
        return a.root == kRootPow ? launch_fwd_t<T, kPow, kRootPow>(a, grid, s)
                                  : launch_fwd_t<T, kPow, kRootNone>(a, grid, s);
    }
}

hipError_t launch_forward(bool f64, int hk, const FwdArgs &a, int grid,
                          hipStream_t s)
{
    return f64 ? launch_fwd_dtype<double>(hk, a, grid, s)
               : launch_fwd_dtype<float>(hk, a, grid, s);
}

template hipError_t launch_pack<float>(const int64_t *, int64_t, const void *,
                                       const void *, unsigned char *, int64_t,
                                       hipStream_t, int64_t);
template hipError_t launch_pack<double>(const int64_t *, int64_t, const void *,
                                        const void *, unsigned char *, int64_t,
                                        hipStream_t, int64_t);
template hipError_t launch_validate<float>(const int64_t *, int64_t,
                                           const void *, const void *,
                                           unsigned char *, int64_t,
                                           hipStream_t);
template hipError_t launch_validate<double>(const int64_t *, int64_t,
                                            const void *, const void *,
                                            unsigned char *, int64_t,
                                            hipStream_t);

}  // namespace pcf

#ifdef PCF_PHASE_TIMING
// Timing builds only: copies out (and with `reset` clears) the per-phase
// cycle sums of the tile kernel (see PhaseClock).
extern "C" int pcf_debug_phase(unsigned long long *host, int reset)
{
    if (hipMemcpyFromSymbol(host, HIP_SYMBOL(pcf::g_phase_cycles),
                            sizeof(pcf::g_phase_cycles)) != hipSuccess)
        return -1;
    if (reset) {
        static const unsigned long long zero[sizeof(pcf::g_phase_cycles) / 8] = {0};
        if (hipMemcpyToSymbol(HIP_SYMBOL(pcf::g_phase_cycles), zero, sizeof(zero)) !=
            hipSuccess)
            return -2;
    }
    return 0;
}
#endif
