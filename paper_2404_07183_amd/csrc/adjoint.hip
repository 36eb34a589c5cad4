// adjoint.hip -- the backward pass of the pairwise matrix: dL/dt and dL/dv
// of every breakpoint for a loss L with dL/dF_ij = G_ij.
//
// The paper only remarks (Section 3, after Algorithm "CombineIntegrate")
// that the integral's parameter derivatives are analytic. Differentiating
// I = sum over cells of h(a, b) * width:
//   dI/dv_f[k] = sum over cells where f takes value v_f[k] of
//                (dh/da)(a, b) * width;
//   dI/dt_f[k] = h(v_f[k-1], g(t_k)) - h(v_f[k], g(t_k))   (k >= 1), with
//                g(t_k) taken just after / just before t_k for the right /
//                left derivative; where g also breaks at t_k the mean of
//                the two one-sided derivatives is used.
// The g side follows from the symmetry of h. The first time and the last
// value of each PCF are fixed parameters (gradient 0). For the L_p distance
// the chain factor dF/dI = (1/p) F^(1-p) is applied (0 when F = 0).
//
// Each pair's merge is recomputed -- the same tiles, the same even split of
// a tile's steps over the lanes and the same merge-path starts as the
// forward kernel -- so nothing is stored between forward and backward. A
// lane keeps the value gradient of its current two pieces in registers and
// adds it to an LDS accumulator (one per breakpoint record of the tile) when
// the piece ends; time gradients go to LDS at each breakpoint. The tile then
// adds its LDS accumulators to dL/dt, dL/dv in HBM with atomics.
#include <hip/hip_runtime.h>

#include <float.h>
#include <math.h>
#include <stdint.h>

#include "common.hpp"
#include "launch.hpp"
#include "tile.hpp"

namespace pcf {

// dh/da at (a, b) for h in {|a-b|, (a-b)^2, ab, |a-b|^p}; sign(0) = 0.
template <int HK>
__device__ __forceinline__ double dhda(double a, double b, double p)
{
    if constexpr (HK == kProd) {
        return b;
    } else {
        const double d = a - b;
        const double s = (d > 0.0) ? 1.0 : ((d < 0.0) ? -1.0 : 0.0);
        if constexpr (HK == kAbs)
            return s;
        else if constexpr (HK == kSqr)
            return 2.0 * d;
        else
            return p * pow(fabs(d), p - 1.0) * s;
    }
}

// Gradient accumulators of one side of a pair: slot q holds (dL/dt, dL/dv)
// of record q -- record q is (t_{k+1}, v_k) of the PCF, so the value
// gradient of piece k goes to slot k and the time gradient of breakpoint
// t_{k+1} goes to slot k + 1. In LDS mode the slots are in LDS next to the
// records; in global mode they are the output arrays themselves, reached
// through the PCF's row base.
struct GradSink {
    double *gt;  // indexed by record index
    double *gv;
    int32_t last;  // record index of the PCF's last row (fixed value)
};

__device__ __forceinline__ void sink_add_t(const GradSink &s, int32_t q, double x)
{
    atomicAdd(&s.gt[q], x);
}
__device__ __forceinline__ void sink_add_v(const GradSink &s, int32_t q, double x)
{
    if (q < s.last)
        atomicAdd(&s.gv[q], x);
}

// Steps [d, d + m) of pair (A, B) with weight W; records from `src` (LDS or
// global), gradients to the two sinks. m is a multiple of kStepBlock.
template <int HK, typename Src>
__device__ __forceinline__ void adjoint_pair(Src src, int32_t A, int32_t na,
                                             int32_t B, int32_t nb, int64_t d,
                                             int64_t m, double W, double p,
                                             const GradSink &sa,
                                             const GradSink &sb)
{
    const double S = sentinel<double>();
    int32_t ia, ib;
    double x;
    pair_start<double>(src, A, na, B, nb, d, ia, ib, x);
    Rec<double> ra = src[ia], rb = src[ib];
    double gva = 0.0, gvb = 0.0;  // value gradients of the current pieces
    for (int64_t q = 0; q < m; ++q) {
        const double y = ra.t <= rb.t ? ra.t : rb.t;
        const double w = y - x;
        gva += dhda<HK>(ra.v, rb.v, p) * w;
        gvb += dhda<HK>(rb.v, ra.v, p) * w;
        if (ra.t <= rb.t) {
            // the row side's breakpoint at y
            const Rec<double> na_ = src[ia + 1];
            if (y < S) {
                double dta;
                if (rb.t == y) {
                    // the column side breaks at y too: mean of the one-sided
                    // derivatives, for both breakpoints (the column side's
                    // own step at y, next, has width 0 and adds nothing)
                    const double bn = src[ib + 1].v;
                    dta = 0.5 * (hval<double, HK>(ra.v, bn, p) - hval<double, HK>(na_.v, bn, p) +
                                 hval<double, HK>(ra.v, rb.v, p) - hval<double, HK>(na_.v, rb.v, p));
                    const double dtb =
                        0.5 * (hval<double, HK>(na_.v, rb.v, p) - hval<double, HK>(na_.v, bn, p) +
                               hval<double, HK>(ra.v, rb.v, p) - hval<double, HK>(ra.v, bn, p));
                    sink_add_t(sb, ib + 1, W * dtb);
                } else {
                    dta = hval<double, HK>(ra.v, rb.v, p) - hval<double, HK>(na_.v, rb.v, p);
                }
                sink_add_t(sa, ia + 1, W * dta);
            }
            sink_add_v(sa, ia, W * gva);
            gva = 0.0;
            ++ia;
            ra = na_;
        } else {
            // the column side's breakpoint at y (strictly before the row
            // side's next one); a width-0 step is the second half of a tie
            // already handled above
            const Rec<double> nb_ = src[ib + 1];
            if (y < S && y > x) {
                const double dtb =
                    hval<double, HK>(ra.v, rb.v, p) - hval<double, HK>(ra.v, nb_.v, p);
                sink_add_t(sb, ib + 1, W * dtb);
            }
            sink_add_v(sb, ib, W * gvb);
            gvb = 0.0;
            ++ib;
            rb = nb_;
        }
        x = y;
    }
    sink_add_v(sa, ia, W * gva);
    sink_add_v(sb, ib, W * gvb);
}

// ---------------------------------------------------------------------------
// The LDS adjoint chain: the forward chain's P/Q formulation (h symmetric,
// P the piece loaded last, Q the other one, one full-wave record read per
// step) with each piece's value-gradient accumulator. LDS record q and its
// two gradient slots belong together, so the slot of a piece is its record
// index and the chain never needs to know which PCF a piece belongs to.
// Fixed parameters (t_0, the last value) and padding slots receive terms
// too; the flush at the end of the tile drops them.
typedef double d2 __attribute__((ext_vector_type(2)));

struct AdjChain {
    d2 P, Q;               // (end time, value) of the two current pieces
    int32_t iP, iQ;        // their record indices (= gradient slots)
    double gP, gQ;         // value gradients of the two pieces so far
    double x;              // start of the current cell
    double W;              // weight of the current pair
    int32_t left;          // steps left in the current pair
    int32_t r, c, rb, rn, cb, cn;
};

__device__ __forceinline__ double adj_min(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double adj_max(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ int32_t adj_pair_steps(int32_t na, int32_t nb)
{
    return (na + nb - 2 + kStepBlock - 1) & ~(kStepBlock - 1);
}

template <int HK>
__device__ __forceinline__ void adj_step(AdjChain &ch, const d2 *lv, double *lgt,
                                         double *lgv, double p)
{
    const double tP = ch.P.x, tQ = ch.Q.x, vP = ch.P.y, vQ = ch.Q.y;
    const double y = adj_min(tP, tQ);
    const double w = y - ch.x;
    ch.x = y;
    ch.gP = fma(dhda<HK>(vP, vQ, p), w, ch.gP);
    ch.gQ = fma(dhda<HK>(vQ, vP, p), w, ch.gQ);
    const bool c = tP <= tQ;
    // E: the piece that ends at y, O: the one that goes on
    const int32_t iE = c ? ch.iP : ch.iQ, iO = c ? ch.iQ : ch.iP;
    const double vE = c ? vP : vQ, vO = c ? vQ : vP;
    const double gE = c ? ch.gP : ch.gQ, gO = c ? ch.gQ : ch.gP;
    const double tO = adj_max(tP, tQ);
    const d2 N = lv[iE + 1];
    atomicAdd(&lgv[iE], ch.W * gE);
    // time gradient of E's breakpoint y (slot iE + 1); a zero-width step is
    // the second half of a tie, handled at the tie
    if (w > 0.0) {
        const double vN = N.y;
        double dE;
        if (tO == y) {
            // O breaks at y too: mean of the one-sided derivatives, for both
            const double vON = lv[iO + 1].y;
            dE = 0.5 * (hval<double, HK>(vE, vON, p) - hval<double, HK>(vN, vON, p) +
                        hval<double, HK>(vE, vO, p) - hval<double, HK>(vN, vO, p));
            const double dO =
                0.5 * (hval<double, HK>(vO, vN, p) - hval<double, HK>(vON, vN, p) +
                       hval<double, HK>(vO, vE, p) - hval<double, HK>(vON, vE, p));
            atomicAdd(&lgt[iO + 1], ch.W * dO);
        } else {
            dE = hval<double, HK>(vE, vO, p) - hval<double, HK>(vN, vO, p);
        }
        atomicAdd(&lgt[iE + 1], ch.W * dE);
    }
    ch.P = N;
    ch.iP = iE + 1;
    ch.gP = 0.0;
    ch.Q.x = tO;
    ch.Q.y = vO;
    ch.iQ = iO;
    ch.gQ = gO;
}

// Starting state at step d of pair k (merge-path split), weight from sh.part.
__device__ __forceinline__ void adj_begin(AdjChain &ch, const TileShared &sh,
                                          const Rec<double> *lrec, int32_t k,
                                          int64_t d, int32_t C)
{
    const d2 *lv = reinterpret_cast<const d2 *>(lrec);
    const int r = div_by_c(k, sh.cmag), c = k - r * C;
    ch.r = r;
    ch.c = c;
    ch.rb = sh.rb[r];
    ch.rn = sh.rn[r];
    ch.cb = sh.cb[c];
    ch.cn = sh.cn[c];
    int32_t i0, j0;
    double x;
    pair_start<double>(lrec, ch.rb, ch.rn, ch.cb, ch.cn, d, i0, j0, x);
    ch.iP = i0;
    ch.iQ = j0;
    ch.P = lv[i0];
    ch.Q = lv[j0];
    ch.x = x;
    ch.gP = 0.0;
    ch.gQ = 0.0;
    ch.W = sh.part[k];
    ch.left = adj_pair_steps(ch.rn, ch.cn) - (int32_t)d;
}

// Next pair with steps (row-major pair order; see chain_next_pair of the
// forward kernel).
__device__ __forceinline__ void adj_next_pair(AdjChain &ch, const TileShared &sh,
                                              const Rec<double> *lrec, int32_t C,
                                              bool diag, int gram)
{
    const d2 *lv = reinterpret_cast<const d2 *>(lrec);
    int32_t r = ch.r, c = ch.c, rb = ch.rb, rn = ch.rn, cb = ch.cb, cn = ch.cn;
    do {
        if (c + 1 < C) {
            cb += cn + kPad;
            ++c;
            cn = sh.cn[c];
        } else {
            rb += rn + kPad;
            ++r;
            rn = sh.rn[r];
            c = diag ? (gram ? r : r + 1) : 0;
            cb = sh.cb[c];
            cn = sh.cn[c];
        }
    } while (adj_pair_steps(rn, cn) == 0);
    ch.r = r;
    ch.c = c;
    ch.rb = rb;
    ch.rn = rn;
    ch.cb = cb;
    ch.cn = cn;
    ch.iP = rb;
    ch.iQ = cb;
    ch.P = lv[rb];
    ch.Q = lv[cb];
    ch.x = 0.0;
    ch.gP = 0.0;
    ch.gQ = 0.0;
    ch.W = sh.part[r * C + c];
    ch.left = adj_pair_steps(rn, cn);
}

template <int HK>
__device__ __forceinline__ void adj_lane_chain(const TileShared &sh,
                                               const Rec<double> *lrec, double *lgt,
                                               double *lgv, int64_t s, int64_t e,
                                               int32_t k, int32_t C, bool diag,
                                               int gram, double p)
{
    const d2 *lv = reinterpret_cast<const d2 *>(lrec);
    AdjChain ch;
    // (an LDS tile: its step prefix is the 32-bit one)
    adj_begin(ch, sh, lrec, k, s - sh.pw[k], C);
    for (int32_t blk = (int32_t)((e - s) / kStepBlock); blk > 0; --blk) {
        if (ch.left == 0) {
            atomicAdd(&lgv[ch.iP], ch.W * ch.gP);
            atomicAdd(&lgv[ch.iQ], ch.W * ch.gQ);
            adj_next_pair(ch, sh, lrec, C, diag, gram);
        }
#pragma unroll
        for (int u = 0; u < kStepBlock; ++u)
            adj_step<HK>(ch, lv, lgt, lgv, p);
        ch.left -= kStepBlock;
    }
    // the pieces going on past this run: their gradients so far
    atomicAdd(&lgv[ch.iP], ch.W * ch.gP);
    atomicAdd(&lgv[ch.iQ], ch.W * ch.gQ);
}

template <int HK>
__global__ __launch_bounds__(kThreads) void pairwise_adjoint_tiles(BwdArgs args)
{
    // tile state in static LDS, records (and the adjoint's accumulators)
    // in the dynamic part: distinct objects, so the compiler knows that the
    // direct record loads into the latter never touch the former
    __shared__ TileShared sh;
    extern __shared__ __align__(16) unsigned char smem[];
    const WsHeader &h = hdr_of(args.ws);
    Rec<double> *lrec = reinterpret_cast<Rec<double> *>(smem);
    int64_t *pw64 = reinterpret_cast<int64_t *>(lrec);  // wide step prefix
    // gradient slots (gt, gv) follow the record slots
    double *lg = reinterpret_cast<double *>(lrec + h.lds_records);
    const Rec<double> *grec = reinterpret_cast<const Rec<double> *>(args.ws + h.off_rec);
    const int64_t *offsets = args.offsets;
    const int tid = threadIdx.x;
    const double p = args.p;

    PhaseClock pc;  // (cycle counters only in timing builds)
    TileLoop loop;
    loop.start<double, true>(sh, args.ws, offsets, lrec, grec);
    while (loop.live(sh, args.ws)) {
        const TileDesc &D = sh.desc[loop.cur];
        const bool gmode = D.global_mode != 0;
        tile_scan<double>(sh, D, args.gram, gmode ? grec : lrec, pw64, pc);
        const int32_t R = D.R, C = D.C, npairs = sh.npairs;
        const bool diag = D.diag != 0;
        const int64_t total = pw_at(sh, pw64, npairs);
        const int64_t nslots = diag ? D.rrecs : D.rrecs + D.crecs;
        if (!gmode)
            for (int64_t q = tid; q < 2 * nslots; q += kThreads)
                lg[q] = 0.0;
        // pair weights: W = (G_ij + G_ji) * chain for i != j, G_ii on the
        // diagonal; stored in the partial-sum slots (unused here)
        if (tid < npairs) {
            const int r = div_by_c(tid, sh.cmag), c = tid - r * C;
            const int64_t i = D.r_lo + r, j = D.c_lo + c;
            double W = 0.0;
            if (pw_at(sh, pw64, tid + 1) > pw_at(sh, pw64, tid)) {
                W = args.grad_out[i * args.ldg + j];
                if (i != j)
                    W += args.grad_out[j * args.ldg + i];
                if (args.chain) {
                    const double F = args.fwd_out[i * args.ldf + j];
                    W = F > 0.0 ? W * (1.0 / p) * pow(F, 1.0 - p) : 0.0;
                }
            }
            sh.part[tid] = W;
        }
        sync_lds();
        loop.take_next(args.ws);

        // this lane's share of the tile's steps
        int64_t s, e;
        lane_steps(sh, tid, total, s, e);
        if (s < e && !gmode) {
            adj_lane_chain<HK>(sh, lrec, lg, lg + nslots, s, e, sh.pairof[tid], C,
                               diag, args.gram, p);
        } else if (s < e) {
            int32_t k = sh.pairof[tid];
            int64_t d = s - pw_at(sh, pw64, k);
            while (s < e) {
                const int r = div_by_c(k, sh.cmag), c = k - r * C;
                const int64_t len = pw_at(sh, pw64, k + 1) - pw_at(sh, pw64, k);
                const int64_t m = (len - d < e - s) ? len - d : e - s;
                const int32_t A = sh.rb[r], B = sh.cb[c];
                GradSink sa, sb;
                sa.last = A + sh.rn[r] - 1;
                sb.last = B + sh.cn[c] - 1;
                if (gmode) {
                    // global record index -> CSR row: row = record - i * kPad
                    const int64_t i = D.r_lo + r, j = D.c_lo + c;
                    sa.gt = args.grad_t - i * kPad;
                    sa.gv = args.grad_v - i * kPad;
                    sb.gt = args.grad_t - j * kPad;
                    sb.gv = args.grad_v - j * kPad;
                    adjoint_pair<HK>(grec, A, sh.rn[r], B, sh.cn[c], d, m,
                                     sh.part[k], p, sa, sb);
                } else {
                    sa.gt = lg;
                    sa.gv = lg + nslots;
                    sb.gt = lg;
                    sb.gv = lg + nslots;
                    adjoint_pair<HK>(lrec, A, sh.rn[r], B, sh.cn[c], d, m,
                                     sh.part[k], p, sa, sb);
                }
                s += m;
                d = 0;
                ++k;
                while (k < npairs && pw_at(sh, pw64, k + 1) == pw_at(sh, pw64, k))
                    ++k;
            }
        }
        sync_lds();
        loop.decode_next(sh, args.ws, offsets);

        // add the tile's accumulators to the outputs; slot 0 of a PCF's
        // time gradient (t_0) and the last value stay untouched (fixed)
        if (!gmode) {
            for (int64_t q = tid; q < nslots; q += kThreads) {
                const bool in_rows = q < D.rrecs;
                const int64_t base = in_rows ? D.rrec0 : D.crec0;
                const int64_t lq = in_rows ? q : q - D.rrecs;
                const int64_t rec = base + lq;           // global record index
                // PCF of this record: the block's PCF whose record range
                // holds it
                const int32_t nb = in_rows ? R : C;
                const int32_t *bs = in_rows ? sh.rb : sh.cb;
                const int32_t *ns = in_rows ? sh.rn : sh.cn;
                const int64_t pcf0 = in_rows ? D.r_lo : D.c_lo;
                // last PCF of the block whose records start at or before q
                int32_t which = 0, hi = nb - 1;
                while (which < hi) {
                    const int32_t mid = (which + hi + 1) >> 1;
                    if (bs[mid] <= q)
                        which = mid;
                    else
                        hi = mid - 1;
                }
                const int64_t kk = q - bs[which];  // record within the PCF
                if (kk >= ns[which])
                    continue;                      // padding
                const int64_t row = rec - (pcf0 + which) * kPad;
                const double gtv = lg[q], gvv = lg[nslots + q];
                if (kk >= 1 && gtv != 0.0)
                    atomicAdd(&args.grad_t[row], gtv);
                if (kk + 1 < ns[which] && gvv != 0.0)
                    atomicAdd(&args.grad_v[row], gvv);
            }
        }
        // (the accumulator flush reads the block metadata)
        loop.stage_next<double, true>(sh, args.ws, grec, offsets, lrec, true);
        loop.advance();
    }
}

// Zero a double array (a kernel, so that captured graphs replay it).
__global__ void zero_doubles(double *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(zero_doubles, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <int HK>
static hipError_t launch_bwd_t(const BwdArgs &a, int grid, hipStream_t s)
{
    const size_t shm = tile_shared_bytes(16, true);
    const hipError_t e = ensure_dynamic_lds(
        reinterpret_cast<const void *>(&pairwise_adjoint_tiles<HK>), (int)shm);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((pairwise_adjoint_tiles<HK>), dim3(grid), dim3(kThreads),
                       shm, s, a);
    return hipGetLastError();
}

hipError_t launch_backward(int hk, const BwdArgs &a, int grid, hipStream_t s)
{
    switch (hk) {
    case kAbs: return launch_bwd_t<kAbs>(a, grid, s);
    case kSqr: return launch_bwd_t<kSqr>(a, grid, s);
    case kProd: return launch_bwd_t<kProd>(a, grid, s);
    default: return launch_bwd_t<kPow>(a, grid, s);
    }
}

}  // namespace pcf
