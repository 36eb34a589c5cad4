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
// the piece ends; time gradients go to LDS at each breakpoint. The
// accumulators are 64-bit fixed point at power-of-two scales bounded per
// tile, so a tile's sums do not depend on the order of its adds. The tile
// then adds them to dL/dt, dL/dv in HBM with atomics of the set's dtype, or,
// for bit-identical results, as 64-bit integers at scales bounded over the
// whole set (in the gradient arrays themselves for FP64, in the workspace
// for FP32), converted by a last pass. FP64 and FP32 sets run the same
// kernel on their own record type.
#include <hip/hip_runtime.h>

#include <float.h>
#include <math.h>
#include <stdint.h>

#include "common.hpp"
#include "launch.hpp"
#include "tile.hpp"

// The device library's maximum over the active lanes of a wave (declared
// here: HIP declares it only with its warp-sync builtins enabled).
extern "C" __device__ __attribute__((const)) double __ockl_wfred_max_f64(double);

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

// ---------------------------------------------------------------------------
// Fixed-point gradient sums. A gradient term w g (w a pair weight already
// multiplied by a power-of-two scale 2^s) is added as the 64-bit integer
// floor(y), y = w g + 1/2: its high word floor(y / 2^32), its low word the
// remainder y - 2^32 floor(y / 2^32), which lies in [0, 2^32) (exact but for
// its own rounding below one unit). So each add is w g within one unit 2^-s,
// or within the FP64 rounding of w g where that is coarser (|y| < 2^62).
// Integer sums are exact modulo 2^64 and do not depend on the order of the
// adds; the scales are chosen from bounds on the terms so that no final sum
// leaves the 64-bit range (partial sums may wrap).
__device__ __forceinline__ long long fixed_of(double w, double g)
{
    const double y = fma(w, g, 0.5);
    const double hi = floor(y * 0x1p-32);
    const double lo = fma(hi, -0x1p32, y);
    return (long long)(((unsigned long long)(unsigned)(int)hi << 32) |
                       (unsigned long long)(unsigned)lo);
}

// The exponent s with B 2^s < 2^target and Wm 2^s <= 2^1000, at least
// -1000 (B > 0; taken as 2^1024 where it overflowed; 0 where B is 0 or NaN,
// whose terms are all 0).
__device__ __forceinline__ int scale_exp(double B, double Wm, int target)
{
    if (!(B > 0.0))
        return 0;
    int e = 1024, ew = 0;
    if (isfinite(B))
        frexp(B, &e);  // B < 2^e
    if (Wm > 0.0)
        frexp(Wm, &ew);
    int sh = target - e;
    sh = sh > 1000 - ew ? 1000 - ew : sh;
    return sh < -1000 ? -1000 : sh;
}

// Bounds on one pair's gradient terms, from the largest |W|, |v| and piece
// length Wm, vm, Lm of the pairs and pieces concerned: a value gradient over
// one piece is at most |W| max|dh/da| times the piece's length (Bv); a time
// gradient is at most 2 |W| max|h| (a jump of h, or the mean of two at a
// tie), and any single add of one is a part of such a term at most twice
// that (Bt = 4 Wm max|h|). (|a - b| <= 2 vm.)
template <int HK>
__device__ __forceinline__ void pair_bounds(double Wm, double vm, double Lm, double p,
                                            double &Bv, double &Bt)
{
    const double a = 2.0 * vm;
    double dh, hm;
    if constexpr (HK == kAbs) {
        dh = 1.0;
        hm = a;
    } else if constexpr (HK == kSqr) {
        dh = 2.0 * a;
        hm = a * a;
    } else if constexpr (HK == kProd) {
        dh = vm;
        hm = vm * vm;
    } else {
        dh = p * pow(a, p - 1.0);
        hm = pow(a, p);
    }
    Bv = Wm * dh * Lm;
    Bt = 4.0 * Wm * hm;
}

// The set's scale exponents of the deterministic adjoint's sums in HBM: a
// breakpoint's gradient sums one term per partner, at most n + 1 of them (a
// diagonal Gram pair adds twice), so (n + 1) B below 2^61 keeps every final
// sum, and the rounding of its adds, inside 64 bits.
template <int HK>
__device__ __forceinline__ void set_exps(const WsHeader &h, int64_t n, double p, int &ev,
                                         int &et)
{
    const double Wm = __longlong_as_double((long long)h.adj_max[0]);
    const double vm = __longlong_as_double((long long)h.adj_max[1]);
    const double Lm = __longlong_as_double((long long)h.adj_max[2]);
    double Bv, Bt;
    pair_bounds<HK>(Wm, vm, Lm, p, Bv, Bt);
    const double m = (double)(n + 1);
    ev = scale_exp(m * Bv, Wm, 61);
    et = scale_exp(m * Bt, Wm, 61);
}

// v 2^-k rounded half up, for a sum v in units 2^-s1 brought to units
// 2^-(s1 - k). (The bounds keep a left shift's result inside 64 bits.)
__device__ __forceinline__ long long fixed_rescale(long long v, int k)
{
    if (k <= 0)
        return k <= -63 ? 0 : (long long)((unsigned long long)v << -k);
    if (k >= 64)
        return 0;
    return (v >> k) + ((v >> (k - 1)) & 1);
}

// Gradient accumulators of one side of a pair: slot q holds (dL/dt, dL/dv)
// of record q -- record q is (t_{k+1}, v_k) of the PCF, so the value
// gradient of piece k goes to slot k and the time gradient of breakpoint
// t_{k+1} goes to slot k + 1. In LDS mode the slots are in LDS next to the
// records; in global mode they are the output arrays themselves, reached
// through the PCF's row base.
template <typename T> struct GradSink {
    T *gt;  // indexed by record index
    T *gv;
    unsigned long long *at, *av;  // fixed-point sums, indexed alike
    int32_t last;  // record index of the PCF's last row (fixed value)
    int fixed;     // 1: add to at, av at scales st, sv instead
    double st, sv;
};

template <typename T>
__device__ __forceinline__ void sink_add_t(const GradSink<T> &s, int32_t q, double x)
{
    if (s.fixed)
        atomicAdd(&s.at[q], (unsigned long long)fixed_of(x, s.st));
    else
        atomicAdd(&s.gt[q], (T)x);
}
template <typename T>
__device__ __forceinline__ void sink_add_v(const GradSink<T> &s, int32_t q, double x)
{
    if (q >= s.last)
        return;
    if (s.fixed)
        atomicAdd(&s.av[q], (unsigned long long)fixed_of(x, s.sv));
    else
        atomicAdd(&s.gv[q], (T)x);
}

// The record at src[i] in FP64 (the sentinel time becomes DBL_MAX).
template <typename T>
__device__ __forceinline__ Rec<double> rec64(const Rec<T> *src, int64_t i)
{
    const Rec<T> r = src[i];
    Rec<double> o;
    o.t = r.t < sentinel<T>() ? (double)r.t : sentinel<double>();
    o.v = (double)r.v;
    return o;
}

// Steps [d, d + m) of pair (A, B) with weight W; records from global
// memory, taken in FP64; gradients to the two sinks. m is a multiple of
// kStepBlock.
template <int HK, typename T>
__device__ __forceinline__ void adjoint_pair(const Rec<T> *src, int32_t A, int32_t na,
                                             int32_t B, int32_t nb, int64_t d,
                                             int64_t m, double W, double p,
                                             const GradSink<T> &sa,
                                             const GradSink<T> &sb)
{
    const double S = sentinel<double>();
    int32_t ia, ib;
    T x0;
    pair_start<T>(src, A, na, B, nb, d, ia, ib, x0);
    double x = x0 < sentinel<T>() ? (double)x0 : S;
    Rec<double> ra = rec64(src, ia), rb = rec64(src, ib);
    double gva = 0.0, gvb = 0.0;  // value gradients of the current pieces
    for (int64_t q = 0; q < m; ++q) {
        const double y = ra.t <= rb.t ? ra.t : rb.t;
        const double w = y - x;
        gva += dhda<HK>(ra.v, rb.v, p) * w;
        gvb += dhda<HK>(rb.v, ra.v, p) * w;
        if (ra.t <= rb.t) {
            // the row side's breakpoint at y
            const Rec<double> na_ = rec64(src, ia + 1);
            if (y < S) {
                double dta;
                if (rb.t == y) {
                    // the column side breaks at y too: mean of the one-sided
                    // derivatives, for both breakpoints (the column side's
                    // own step at y, next, has width 0 and adds nothing)
                    const double bn = (double)src[ib + 1].v;
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
            const Rec<double> nb_ = rec64(src, ib + 1);
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
// The LDS adjoint chain: the forward chain's P/Q formulation and record walk
// (h symmetric, P the piece loaded last, Q the other one, one record read
// per step) with each piece's value-gradient accumulator, in the set's
// precision T; the gradient sums are fixed point (lds_add).
//
// Gradient slots: record q (at LDS address R0 + Rq, R = 16 bytes for FP64
// records, 8 for FP32) has two 64-bit slots, dL/dv of its piece at V0 + 8q
// and dL/dt of its end time AdjLayout<T>::kGt bytes further, so the slots of
// a piece are found from its record address alone (a shift by
// log2(R / 8) and the add of a workgroup constant, V0 - R0 8 / R) and the
// chain never needs to know which PCF a piece belongs to. Each step ends one
// piece E: its value gradient so far and the time gradient of its end time y
// go to E's slots (two LDS atomic adds at the walk's address, immediate
// offsets). Fixed parameters (the last value, the sentinel end time of the
// last piece) and padding slots receive terms too; the flush at the end of
// the tile drops them.
//
// Time gradient at a breakpoint y where E ends and the other piece O goes
// on: h(vE, vO) - h(vN, vO), vN the value after y. Where O breaks at y too
// (equal times: P ends, as P wins ties), the mean of the one-sided
// derivatives is taken for both breakpoints in that step, reading O's next
// value; the next step, which ends O with width 0, adds no time gradient.
typedef double d2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) long long lds_i64;

// The adjoint's tile state: its partial-sum slots hold the pair weights.
using AdjShared = TileSharedT<kMaxPairs>;
static_assert(sizeof(AdjShared) + kAdjLdsBytes <= 160 * 1024 / kWgPerCu,
              "the adjoint's tile state and records must fit a CU's LDS");
static_assert((int64_t)kMaxBlock * (kAdjLdsBytes / 8) + 8 * (int64_t)kMaxPairs <
                  ((int64_t)1 << 30),
              "adjoint LDS tiles scan in 32 bits");

// The adjoint's LDS layout for records of type T.
template <typename T> struct AdjLayout {
    static constexpr int kRecBytes = (int)sizeof(Rec<T>);
    static constexpr int kRecords = adj_lds_records(kRecBytes);  // records a tile
    static constexpr uint32_t kGt = adj_gt_offset(kRecBytes);    // dL/dv -> dL/dt slot
    static constexpr int kUnroll = adj_stage_unroll(kRecBytes);  // staging, per thread
    static constexpr int kShift = kRecBytes == 16 ? 1 : 0;       // record -> slot address
    static_assert(kRecBytes == 16 || kRecBytes == 8, "record size");
};

template <typename T> struct AdjChain {
    typedef typename RecVec<T>::type V;
    V P;                   // (end time, value) of the piece loaded last
    uint32_t gb;           // gradient slot base (workgroup constant)
    T tQ, vQ;              // the other piece
    LdsWalk<T> w;          // record addresses
    T gQ;                  // value gradient of Q so far, in units of
                           // gunit<HK> (P's is 0: loaded by the last step)
    T x;                   // start of the current cell
    double Wv, Wt;         // pair weight times the unit of dh/da; pair weight
                           // (times the tile's value and time slot scales)
    double sv, st;         // the tile's slot scales
    int32_t left;          // steps left in the current pair
    int32_t k, r, c, rb, rn, cb, cn;
};

// dh/da(a, b) = gunit * dP(a, b); dh/da(b, a) = gunit * dQ(a, b).
template <int HK>
__device__ __forceinline__ double gunit(double p)
{
    if constexpr (HK == kSqr)
        return 2.0;
    else if constexpr (HK == kAbs || HK == kProd)
        return 1.0;
    else
        return p;
}

// h(e, o) - h(n, o)
template <typename T, int HK>
__device__ __forceinline__ T hdiff(T e, T n, T o, T p)
{
    if constexpr (HK == kSqr)
        return (e - n) * ((e + n) - T(2) * o);
    else if constexpr (HK == kProd)
        return (e - n) * o;
    else
        return hval<T, HK>(e, o, p) - hval<T, HK>(n, o, p);
}

// The step's value-gradient terms, dh/da(a, b) = gunit * dP and
// dh/da(b, a) = gunit * dQ, and h(a, b), from the one difference d = a - b
// (|d|^p = |d|^(p-1) |d| for general p).
template <typename T, int HK>
__device__ __forceinline__ void step_terms(T a, T b, T p, T &dP, T &dQ, T &hab)
{
    if constexpr (HK == kProd) {
        dP = b;
        dQ = a;
        hab = a * b;
    } else {
        const T d = a - b;
        if constexpr (HK == kSqr) {
            dP = d;
            hab = d * d;
        } else if constexpr (HK == kAbs) {
            dP = d > T(0) ? T(1) : (d < T(0) ? T(-1) : T(0));
            hab = fabs(d);
        } else {
            const T m = hval<T, HK>(d, T(0), p - T(1));  // |d|^(p-1)
            dP = d > T(0) ? m : (d < T(0) ? -m : T(0));
            hab = m * fabs(d);
        }
        dQ = -dP;
    }
}

// The dL/dv slot of the record at LDS address a, plus Extra bytes (the
// dL/dt slot at Extra + kGt). Extra becomes a constant offset of the atomic.
template <typename T, uint32_t Extra>
__device__ __forceinline__ lds_f64 *grad_slot(uint32_t a, uint32_t gb)
{
    return (lds_f64 *)(size_t)((a >> AdjLayout<T>::kShift) + gb + Extra);
}

// LDS slot add: w g to the nearest unit of the tile's fixed point (w carries
// the tile's scale). Integer LDS atomics are faster than FP64 ones; the adds
// are exact modulo 2^64, so a tile's sums do not depend on their order.
__device__ __forceinline__ void lds_add(lds_f64 *p, double w, double g)
{
    __hip_atomic_fetch_add((lds_i64 *)p, fixed_of(w, g), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One step: the cell [x, y) closes, E (the piece ending at y, P on equal
// times) adds its value gradient and the time gradient of y to its slots.
// h(vE, vO) = h(vP, vQ) by symmetry, so E's own value is needed only in the
// tie branch (where E = P). At a tie the first step adds the mean one-sided
// derivatives of both breakpoints and carries O's next value vON as Q's
// value: the second, width-0 step (which ends O) then adds
// h(vN, vON) - h(vON, vN) = 0 to O's time slot and nothing to any value
// gradient, and O's value is not used after it. A run that begins with such
// a second half subtracts that step's own term at its start (adj_begin).
// Width-0 steps past the sentinel only reach dropped slots.
template <typename T, int K, int HK>
__device__ __forceinline__ void adj_step(AdjChain<T> &ch, T p)
{
    typedef typename RecVec<T>::type V;
    typedef const __attribute__((address_space(3))) V *lds_v;
    constexpr uint32_t kGt = AdjLayout<T>::kGt;
    const T S = sentinel<T>();
    const T tP = ch.P.x, vP = ch.P.y, tQ = ch.tQ, vQ = ch.vQ;
    const T y = min_raw(tP, tQ);
    const T w = y - ch.x;
    ch.x = y;
    T dP, dQ, hPQ;
    step_terms<T, HK>(vP, vQ, p, dP, dQ, hPQ);
    const T gP = dP * w;  // P was loaded by the previous step
    const T gQ = fma(dQ, w, ch.gQ);
    const bool c = tP <= tQ;
    const T vO = c ? vQ : vP;
    const T gE = c ? gP : gQ, gO = c ? gQ : gP;
    const uint32_t aQ = ch.w.S - ch.w.q;  // Q's record address at this step
    const V N = ch.w.template advance<K>(c);
    // E's record address is the walk's q plus K records
    lds_add(grad_slot<T, K * 8>(ch.w.q, ch.gb), ch.Wv, (double)gE);
    T dE = hPQ - hval<T, HK>(N.y, vO, p);
    T vOc = vO;
    if (tP == tQ && y < S) {
        // both break at y (E = P, O = Q): the mean of the one-sided
        // derivatives for both
        const T vON = ((lds_v)(size_t)(aQ + (uint32_t)sizeof(Rec<T>)))->y;
        dE = T(0.5) * (dE + hdiff<T, HK>(vP, N.y, vON, p));
        const T dO = T(0.5) * (hdiff<T, HK>(vQ, vON, vP, p) + hdiff<T, HK>(vQ, vON, N.y, p));
        lds_add(grad_slot<T, kGt>(aQ, ch.gb), ch.Wt, (double)dO);
        vOc = vON;
    }
    lds_add(grad_slot<T, K * 8 + kGt>(ch.w.q, ch.gb), ch.Wt, (double)dE);
    ch.P = N;
    ch.tQ = max_raw(tP, tQ);
    ch.vQ = vOc;
    ch.gQ = gO;
}

template <typename T, int HK, int... Ks>
__device__ __forceinline__ void adj_block(AdjChain<T> &ch, T p,
                                          std::integer_sequence<int, Ks...>)
{
    (adj_step<T, Ks, HK>(ch, p), ...);
    ch.w.end_block();
}

// The value gradients of the two current pieces (at a block boundary, where
// the walk's q is P's record address).
template <typename T>
__device__ __forceinline__ void adj_flush(const AdjChain<T> &ch)
{
    // P's is 0 (just loaded)
    lds_add(grad_slot<T, 0>(ch.w.S - ch.w.q, ch.gb), ch.Wv, (double)ch.gQ);
}

__device__ __forceinline__ int32_t adj_pair_steps(int32_t na, int32_t nb)
{
    return (na + nb - 2 + kStepBlock - 1) & ~(kStepBlock - 1);
}

template <typename T>
__device__ __forceinline__ void adj_load(AdjChain<T> &ch, const Rec<T> *lrec, int32_t iP,
                                         int32_t iQ)
{
    ch.w.set(lrec, iP, iQ);
    ch.P = LdsWalk<T>::at(lrec, iP);
    const typename RecVec<T>::type Q = LdsWalk<T>::at(lrec, iQ);
    ch.tQ = Q.x;
    ch.vQ = Q.y;
    ch.gQ = T(0);
}

// Starting state at step d of pair k (merge-path split), weights from
// sh.part.
template <typename T, int HK>
__device__ __forceinline__ void adj_begin(AdjChain<T> &ch, const AdjShared &sh,
                                          const Rec<T> *lrec, int32_t k, int64_t d,
                                          int32_t C, T p)
{
    typedef typename RecVec<T>::type V;
    typedef const __attribute__((address_space(3))) V *lds_v;
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
    pair_start<T>(lrec, ch.rb, ch.rn, ch.cb, ch.cn, d, i0, j0, x);
    adj_load<T>(ch, lrec, i0, j0);
    ch.x = x;
    ch.Wt = sh.part[k] * ch.st;
    ch.Wv = sh.part[k] * gunit<HK>((double)p) * ch.sv;
    ch.left = adj_pair_steps(ch.rn, ch.cn) - (int32_t)d;
    if (x > T(0) && x < sentinel<T>() && min_raw(ch.P.x, ch.tQ) == x) {
        // the run starts at the width-0 second half of a tie, whose time
        // gradients the run before added in full: this step's own term
        // (as adj_step computes it) is subtracted in advance
        const bool c0 = ch.P.x <= ch.tQ;
        const uint32_t aE = c0 ? ch.w.q : ch.w.S - ch.w.q;
        const T vO0 = c0 ? ch.vQ : ch.P.y;
        const T vN0 = ((lds_v)(size_t)(aE + (uint32_t)sizeof(Rec<T>)))->y;
        T dP, dQ, hPQ;
        step_terms<T, HK>(ch.P.y, ch.vQ, p, dP, dQ, hPQ);
        const T dE = hPQ - hval<T, HK>(vN0, vO0, p);
        lds_add(grad_slot<T, AdjLayout<T>::kGt>(aE, ch.gb), -ch.Wt, (double)dE);
    }
}

// Next pair with steps (row-major pair order, as the forward chain).
template <typename T, int HK>
__device__ __forceinline__ void adj_next_pair(AdjChain<T> &ch, const AdjShared &sh,
                                              const Rec<T> *lrec, int32_t C, bool diag,
                                              int gram, T p)
{
    int32_t k = ch.k, r = ch.r, c = ch.c, rb = ch.rb, rn = ch.rn, cb = ch.cb, cn = ch.cn;
    do {
        ++k;
        if (c + 1 < C) {
            cb += cn + kPad;
            ++c;
            cn = sh.cn[c];
        } else {
            rb += rn + kPad;
            ++r;
            rn = sh.rn[r];
            c = diag ? (gram ? r : r + 1) : 0;
            k = r * C + c;
            cb = sh.cb[c];
            cn = sh.cn[c];
        }
    } while (adj_pair_steps(rn, cn) == 0);
    ch.k = k;
    ch.r = r;
    ch.c = c;
    ch.rb = rb;
    ch.rn = rn;
    ch.cb = cb;
    ch.cn = cn;
    adj_load<T>(ch, lrec, rb, cb);
    ch.x = T(0);
    ch.Wt = sh.part[k] * ch.st;
    ch.Wv = sh.part[k] * gunit<HK>((double)p) * ch.sv;
    ch.left = adj_pair_steps(rn, cn);
}

template <typename T, int HK>
__device__ __forceinline__ void adj_lane_chain(const AdjShared &sh, const Rec<T> *lrec,
                                               uint32_t gb, double sv, double st, int64_t s,
                                               int64_t e, int32_t k, int32_t C, bool diag,
                                               int gram, T p)
{
    AdjChain<T> ch;
    ch.gb = gb;
    ch.sv = sv;
    ch.st = st;
    // (an LDS tile: its step prefix is the 32-bit one)
    adj_begin<T, HK>(ch, sh, lrec, k, s - sh.pw[k], C, p);
    for (int32_t blk = (int32_t)((e - s) / kStepBlock); blk > 0; --blk) {
        if (ch.left == 0) {
            adj_flush(ch);
            adj_next_pair<T, HK>(ch, sh, lrec, C, diag, gram, p);
        }
        adj_block<T, HK>(ch, p, std::make_integer_sequence<int, kStepBlock>{});
        ch.left -= kStepBlock;
    }
    // the piece going on past this run: its gradient so far
    adj_flush(ch);
}

template <typename T, int HK>
__global__ __launch_bounds__(kThreads) void pairwise_adjoint_tiles(BwdArgs args)
{
    typedef AdjLayout<T> L;
    // tile state in static LDS, records (and the adjoint's accumulators)
    // in the dynamic part: distinct objects, so the compiler knows that the
    // direct record loads into the latter never touch the former
    __shared__ AdjShared sh;
    extern __shared__ __align__(16) unsigned char smem[];
    const WsHeader &h = hdr_of(args.ws);
    Rec<T> *lrec = reinterpret_cast<Rec<T> *>(smem);
    int64_t *pw64 = reinterpret_cast<int64_t *>(lrec);  // wide step prefix
    // gradient slots follow the records: dL/dv of record q at lg[q], dL/dt
    // of its end time at lg[L::kRecords + q] (L::kRecords records a tile),
    // as 64-bit fixed-point sums at the tile's scales (lds_add)
    double *lg = reinterpret_cast<double *>(lrec + L::kRecords);
    const uint32_t gb = lds_address(lg) - (lds_address(lrec) >> L::kShift);
    const Rec<T> *grec = reinterpret_cast<const Rec<T> *>(args.ws + h.off_rec);
    const int64_t *offsets = args.offsets;
    const int tid = threadIdx.x;
    const double p = args.p;
    T *const grad_t = reinterpret_cast<T *>(args.grad_t);
    T *const grad_v = reinterpret_cast<T *>(args.grad_v);
    // deterministic mode's 64-bit sums: FP64 gradients hold them in place,
    // FP32 ones in the workspace (dL/dt rows, then dL/dv rows)
    unsigned long long *const acc_t =
        sizeof(T) == 8 ? reinterpret_cast<unsigned long long *>(args.grad_t)
                       : reinterpret_cast<unsigned long long *>(args.ws + h.off_acc);
    unsigned long long *const acc_v =
        sizeof(T) == 8 ? reinterpret_cast<unsigned long long *>(args.grad_v)
                       : acc_t + (h.rec_count - h.npcf * kPad);
    // deterministic mode: the set's scales of the sums in HBM
    int gev = 0, get = 0;
    if (args.fixed)
        set_exps<HK>(h, args.n, p, gev, get);
    const double gsv = ldexp(1.0, gev), gst = ldexp(1.0, get);

    PhaseClock pc;  // (cycle counters only in timing builds)
    TileLoop loop;
    // (direct staging moves 16-byte records)
    loop.start<T, sizeof(Rec<T>) == 16>(sh, args.ws, offsets, lrec, grec);
    pc.mark(-1);
    while (loop.live(sh, args.ws)) {
        const TileDesc &D = sh.desc[loop.cur];
        const bool gmode = D.global_mode != 0;
        tile_scan<T, kWeightsAdjoint>(sh, D, args.gram, gmode ? grec : lrec, pw64, pc);
        const int32_t R = D.R, C = D.C, npairs = sh.npairs;
        const bool diag = D.diag != 0;
        const int64_t total = pw_at(sh, pw64, npairs);
        pc.mark(kPhaseScan);
        pc.tile(total);
        const int64_t nslots = diag ? D.rrecs : D.rrecs + D.crecs;
        if (!gmode)
            for (int64_t q = tid; q < nslots; q += kThreads) {
                lg[q] = 0.0;
                lg[L::kRecords + q] = 0.0;
            }
        // pair weights: W = (G_ij + G_ji) * chain for i != j, G_ii on the
        // diagonal; stored in the partial-sum slots (unused here)
        double mw = 0.0, mv = 0.0, ml = 0.0;  // this thread's largest |W|, |v|, piece
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
            mw = fabs(W);
        }
        if (!gmode) {
            const T S = sentinel<T>();
            for (int64_t q = tid; q < nslots; q += kThreads) {
                const Rec<T> rq = lrec[q];
                mv = fmax(mv, fabs((double)rq.v));
                // a piece starts at the previous record's end time, or at 0
                // where that record is a sentinel (a PCF's first piece: the
                // record before it ends the previous PCF, or pads, or q
                // starts a block)
                const T t0 = (q == 0 || q == D.rrecs) ? T(0) : lrec[q - 1].t;
                if (rq.t < S)
                    ml = fmax(ml, (double)rq.t - (t0 < S ? (double)t0 : 0.0));
            }
            // the tile's maxima through the wave's lanes (every lane is
            // active here), then one slot per wave (the tail-rule values of
            // the scan, unused by the adjoint). The general-p kernel keeps the
            // shuffle butterfly: it is the most register-bound instantiation,
            // and its code stays as tested.
            if constexpr (HK == kPow) {
                for (int h = 32; h >= 1; h >>= 1) {
                    mw = fmax(mw, __shfl_xor(mw, h, 64));
                    mv = fmax(mv, __shfl_xor(mv, h, 64));
                    ml = fmax(ml, __shfl_xor(ml, h, 64));
                }
            } else {
                mw = __ockl_wfred_max_f64(mw);
                mv = __ockl_wfred_max_f64(mv);
                ml = __ockl_wfred_max_f64(ml);
            }
            if ((tid & 63) == 0) {
                sh.rlast[tid >> 6] = mw;
                sh.rlast[16 + (tid >> 6)] = mv;
                sh.clast[tid >> 6] = ml;
            }
        }
        sync_lds();
        loop.take_next(args.ws);
        // the tile's slot scales 2^ev, 2^et. A kept slot sums, over at most
        // 32 partners of its PCF (33 terms: a diagonal Gram pair adds
        // twice), one pair's gradient each, within the pair bounds of the
        // tile's largest |W|, |v| and piece length; each bound below 2^57
        // keeps the slot's final sum below 33 * 2^57 < 2^63. Slots of the
        // fixed last value and of padding may take larger adds; they are
        // dropped.
        int ev = 0, et = 0;
        if (!gmode) {
            double Wm = 0.0, vm = 0.0, Lm = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) {
                Wm = fmax(Wm, sh.rlast[w]);
                vm = fmax(vm, sh.rlast[16 + w]);
                Lm = fmax(Lm, sh.clast[w]);
            }
            double Bv, Bt;
            pair_bounds<HK>(Wm, vm, Lm, p, Bv, Bt);
            ev = scale_exp(Bv, Wm, 57);
            et = scale_exp(Bt, Wm, 57);
        }
        const double sv = ldexp(1.0, ev), st = ldexp(1.0, et);
        const double isv = ldexp(1.0, -ev), ist = ldexp(1.0, -et);
        pc.mark(kPhaseStart);

        // this lane's share of the tile's steps
        int64_t s, e;
        lane_steps(sh, tid, total, s, e);
        if (s < e && !gmode) {
            adj_lane_chain<T, HK>(sh, lrec, gb, sv, st, s, e, sh.pairof[tid], C, diag,
                                  args.gram, (T)p);
        } else if (s < e) {
            int32_t k = sh.pairof[tid];
            int64_t d = s - pw_at(sh, pw64, k);
            while (s < e) {
                const int r = div_by_c(k, sh.cmag), c = k - r * C;
                const int64_t len = pw_at(sh, pw64, k + 1) - pw_at(sh, pw64, k);
                const int64_t m = (len - d < e - s) ? len - d : e - s;
                const int32_t A = sh.rb[r], B = sh.cb[c];
                // global record index -> CSR row: row = record - i * kPad
                const int64_t i = D.r_lo + r, j = D.c_lo + c;
                GradSink<T> sa, sb;
                sa.last = A + sh.rn[r] - 1;
                sb.last = B + sh.cn[c] - 1;
                sa.gt = grad_t - i * kPad;
                sa.gv = grad_v - i * kPad;
                sb.gt = grad_t - j * kPad;
                sb.gv = grad_v - j * kPad;
                sa.at = acc_t - i * kPad;
                sa.av = acc_v - i * kPad;
                sb.at = acc_t - j * kPad;
                sb.av = acc_v - j * kPad;
                sa.fixed = sb.fixed = args.fixed;
                sa.st = sb.st = gst;
                sa.sv = sb.sv = gsv;
                adjoint_pair<HK, T>(grec, A, sh.rn[r], B, sh.cn[c], d, m, sh.part[k], p, sa, sb);
                s += m;
                d = 0;
                ++k;
                while (k < npairs && pw_at(sh, pw64, k + 1) == pw_at(sh, pw64, k))
                    ++k;
            }
        }
        pc.mark(kPhaseMerge);
        // the next tile's staging loads, issued as soon as this wave's merge
        // work is done (into registers: the records are stored to LDS after
        // the accumulator flush, which reads the current block metadata)
        const bool has_next = loop.has_next(sh, args.ws);
        StageRegs<T, false, L::kUnroll> next;
        if (has_next)
            stage_load<T, false, L::kUnroll>(next, sh.desc[loop.nxt()], grec, offsets, lrec);
        sync_lds();
        pc.mark(kPhaseMergeWait);
        loop.decode_next(sh, args.ws, offsets);
        pc.mark(kPhaseStageIssue);

        // the tile's accumulators, read before the next tile's block
        // metadata is stored and added to the outputs after it (so that the
        // staging's wait for its loads does not also wait for these atomics);
        // t_0 and the last value of each PCF stay untouched (fixed). A slot
        // q holds record q's value gradient and its end time's gradient.
        static_assert(L::kUnroll * kThreads >= L::kRecords, "slots per thread");
        double fv[L::kUnroll], ft[L::kUnroll];
        int64_t frow[L::kUnroll];
#pragma unroll
        for (int u = 0; u < L::kUnroll; ++u) {
            const int64_t q = tid + u * kThreads;
            frow[u] = -1;
            fv[u] = ft[u] = 0.0;
            if (gmode || q >= nslots)
                continue;
            const bool in_rows = q < D.rrecs;
            const int64_t base = in_rows ? D.rrec0 : D.crec0;
            const int64_t lq = in_rows ? q : q - D.rrecs;
            const int64_t rec = base + lq;  // global record index
            // PCF of this record: the last PCF of its block whose records
            // start at or before q
            const int32_t nb = in_rows ? R : C;
            const int32_t *bs = in_rows ? sh.rb : sh.cb;
            const int32_t *ns = in_rows ? sh.rn : sh.cn;
            const int64_t pcf0 = in_rows ? D.r_lo : D.c_lo;
            int32_t which = 0;
            if constexpr (HK == kPow) {
                // (the general-p kernels keep their tested code)
                int32_t hi = nb - 1;
                while (which < hi) {
                    const int32_t mid = (which + hi + 1) >> 1;
                    if (bs[mid] <= q)
                        which = mid;
                    else
                        hi = mid - 1;
                }
            } else {
                // five fixed steps (nb <= 32): straight-line code, so the
                // searches of a thread's slots overlap
                static_assert(kMaxBlock <= 32, "lifting steps");
#pragma unroll
                for (int32_t st = 16; st > 0; st >>= 1) {
                    const int32_t j = which + st;
                    if (j < nb && bs[j] <= q)
                        which = j;
                }
            }
            const int64_t kk = q - bs[which];  // record within the PCF
            // padding, and the last record (fixed value, sentinel end time)
            if (kk + 1 >= ns[which])
                continue;
            frow[u] = rec - (pcf0 + which) * kPad;
            const long long *li = reinterpret_cast<const long long *>(lg);
            if (args.fixed) {
                // the sums in the set's units (bit patterns in fv, ft)
                fv[u] = __longlong_as_double(fixed_rescale(li[q], ev - gev));
                ft[u] = __longlong_as_double(fixed_rescale(li[L::kRecords + q], et - get));
            } else {
                fv[u] = (double)li[q] * isv;
                ft[u] = (double)li[L::kRecords + q] * ist;
            }
        }
        pc.mark(kPhaseFinish);
        if (has_next) {
            sync_lds();  // (the slot reads above use the block metadata)
            stage_store<T, false, L::kUnroll>(sh, next, sh.desc[loop.nxt()], lrec);
        }
#pragma unroll
        for (int u = 0; u < L::kUnroll; ++u) {
            if (frow[u] < 0)
                continue;
            if (args.fixed) {
                const unsigned long long bv = (unsigned long long)__double_as_longlong(fv[u]);
                const unsigned long long bt = (unsigned long long)__double_as_longlong(ft[u]);
                if (bv != 0)
                    atomicAdd(&acc_v[frow[u]], bv);
                if (bt != 0)
                    atomicAdd(&acc_t[frow[u] + 1], bt);
                continue;
            }
            if (fv[u] != 0.0)
                atomicAdd(&grad_v[frow[u]], (T)fv[u]);
            if (ft[u] != 0.0)
                atomicAdd(&grad_t[frow[u] + 1], (T)ft[u]);  // the piece's end time
        }
        pc.mark(kPhaseStageStore);
        loop.advance();
        pc.mark(kPhaseAdvance);
    }
    pc.flush((tid & 63) == 0 ? tid >> 6 : -1);
}

#ifdef PCF_PHASE_TIMING
// Timing builds only: the adjoint kernel's per-phase cycle sums (its own
// copy of the counters), as pcf_debug_phase.
extern "C" int pcf_debug_phase_adjoint(unsigned long long *host, int reset)
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

// Zero an array (a kernel, so that captured graphs replay it).
template <typename U> __global__ void zero_array(U *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = U(0);
}

template <typename U> static hipError_t launch_zero_t(U *p, int64_t n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(zero_array<U>, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t s) { return launch_zero_t(p, n, s); }
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s) { return launch_zero_t(p, n, s); }

// ---------------------------------------------------------------------------
// Deterministic adjoint: the set's bounds, then the conversion of its sums.

// Largest value over the block into *dst (bit patterns of non-negative
// doubles order like the doubles).
__device__ __forceinline__ void block_max_to(double m, unsigned long long *dst, double *red)
{
    for (int hop = 32; hop >= 1; hop >>= 1)
        m = fmax(m, __shfl_xor(m, hop, 64));
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0)
        red[w] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < nw; ++k)
            m = fmax(m, red[k]);
        if (m > 0.0)
            atomicMax(dst, (unsigned long long)__double_as_longlong(m));
    }
}

// The largest |W| of the pairs (i, j), i <= j, of a 32 x 32 block of the
// matrix above the diagonal (W as the adjoint kernel forms it; the chain
// factor taken from F_ij and F_ji alike, whichever the tile reads). G_ji
// comes through an LDS transpose so that both reads are coalesced.
__global__ __launch_bounds__(256) void adj_bounds_pairs(BwdArgs a)
{
    __shared__ double gT[32][33], fT[32][33];
    __shared__ double red[4];
    const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
    if (i0 > j0)
        return;  // (the whole block)
    WsHeader *h = reinterpret_cast<WsHeader *>(a.ws);
    const int64_t n = a.n;
    const int c = threadIdx.x & 31, r0 = threadIdx.x >> 5;
    for (int r = r0; r < 32; r += 8) {
        const int64_t j = j0 + r, i = i0 + c;
        const bool in = i < n && j < n;
        gT[r][c] = in ? a.grad_out[j * a.ldg + i] : 0.0;
        fT[r][c] = (in && a.chain) ? a.fwd_out[j * a.ldf + i] : 0.0;
    }
    __syncthreads();
    double m = 0.0;
    for (int r = r0; r < 32; r += 8) {
        const int64_t i = i0 + r, j = j0 + c;
        if (i >= n || j >= n || i > j || (i == j && !a.gram))
            continue;
        double W = a.grad_out[i * a.ldg + j];
        if (i != j)
            W += gT[c][r];
        if (a.chain) {
            const double F1 = a.fwd_out[i * a.ldf + j], F2 = fT[c][r];
            const double W1 = F1 > 0.0 ? W * (1.0 / a.p) * pow(F1, 1.0 - a.p) : 0.0;
            const double W2 = F2 > 0.0 ? W * (1.0 / a.p) * pow(F2, 1.0 - a.p) : 0.0;
            W = fmax(fabs(W1), fabs(W2));
        }
        m = fmax(m, fabs(W));
    }
    block_max_to(m, &h->adj_max[0], red);
}

// The largest |v| and piece length of the packed records (a piece starts
// at the previous record's end time, or at 0 after a sentinel).
template <typename T>
__global__ __launch_bounds__(256) void adj_bounds_records(BwdArgs a)
{
    __shared__ double red[4];
    WsHeader *h = reinterpret_cast<WsHeader *>(a.ws);
    const Rec<T> *rec = reinterpret_cast<const Rec<T> *>(a.ws + h->off_rec);
    const int64_t count = h->rec_count;
    const T S = sentinel<T>();
    double mv = 0.0, ml = 0.0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < count;
         q += (int64_t)gridDim.x * blockDim.x) {
        const Rec<T> r = rec[q];
        mv = fmax(mv, fabs((double)r.v));
        if (r.t < S) {
            const T t0 = q > 0 ? rec[q - 1].t : T(0);
            ml = fmax(ml, (double)r.t - (t0 < S ? (double)t0 : 0.0));
        }
    }
    block_max_to(mv, &h->adj_max[1], red);
    __syncthreads();  // (red is reused)
    block_max_to(ml, &h->adj_max[2], red);
}

// Clears an FP32 plan's 64-bit sums (n words at the header's off_acc).
__global__ __launch_bounds__(256) void adj_zero_acc(unsigned char *ws, int64_t n)
{
    const WsHeader *h = reinterpret_cast<const WsHeader *>(ws);
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(ws + h->off_acc);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        acc[k] = 0ull;
}

hipError_t launch_adj_bounds(bool f64, const BwdArgs &a, hipStream_t s)
{
    hipError_t e = launch_zero(reinterpret_cast<double *>(
                                   a.ws + offsetof(WsHeader, adj_max)),
                               3, s);
    if (e != hipSuccess)
        return e;
    const int64_t nb = (a.n + 31) / 32;
    if (nb > 65535)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(adj_bounds_pairs, dim3((unsigned)nb, (unsigned)nb), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (f64)
        hipLaunchKernelGGL(adj_bounds_records<double>, dim3(1024), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(adj_bounds_records<float>, dim3(1024), dim3(256), 0, s, a);
    return hipGetLastError();
}

// The fixed-point sums (P rows each; FP64 gradients hold them in place,
// FP32 ones in the workspace) to the gradients' type.
template <typename T, int HK>
__global__ __launch_bounds__(256) void adj_finish(BwdArgs a, int64_t P)
{
    const WsHeader &h = *reinterpret_cast<const WsHeader *>(a.ws);
    int ev, et;
    set_exps<HK>(h, a.n, a.p, ev, et);
    const double iv = ldexp(1.0, -ev), it = ldexp(1.0, -et);
    const long long *gt = reinterpret_cast<const long long *>(
        sizeof(T) == 8 ? (const unsigned char *)a.grad_t : a.ws + h.off_acc);
    const long long *gv = reinterpret_cast<const long long *>(
        sizeof(T) == 8 ? (const unsigned char *)a.grad_v : a.ws + h.off_acc + 8 * P);
    T *ot = reinterpret_cast<T *>(a.grad_t);
    T *ov = reinterpret_cast<T *>(a.grad_v);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < P;
         k += (int64_t)gridDim.x * blockDim.x) {
        // (read both sums before writing: FP64 converts in place)
        const long long xt = gt[k], xv = gv[k];
        ot[k] = (T)((double)xt * it);
        ov[k] = (T)((double)xv * iv);
    }
}

template <typename T>
static void launch_finish_t(int hk, const BwdArgs &a, int64_t P, dim3 g, dim3 b, hipStream_t s)
{
    switch (hk) {
    case kAbs: hipLaunchKernelGGL((adj_finish<T, kAbs>), g, b, 0, s, a, P); break;
    case kSqr: hipLaunchKernelGGL((adj_finish<T, kSqr>), g, b, 0, s, a, P); break;
    case kProd: hipLaunchKernelGGL((adj_finish<T, kProd>), g, b, 0, s, a, P); break;
    default: hipLaunchKernelGGL((adj_finish<T, kPow>), g, b, 0, s, a, P); break;
    }
}

hipError_t launch_adj_finish(int hk, bool f64, const BwdArgs &a, int64_t P, hipStream_t s)
{
    if (P <= 0)
        return hipSuccess;
    int64_t blocks = (P + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    const dim3 g((unsigned)blocks), b(256);
    if (f64) {
        launch_finish_t<double>(hk, a, P, g, b, s);
    } else {
        // the FP32 plan's sums are cleared before the adjoint (launch_adj_acc)
        launch_finish_t<float>(hk, a, P, g, b, s);
    }
    return hipGetLastError();
}

hipError_t launch_adj_acc(const BwdArgs &a, int64_t P, hipStream_t s)
{
    if (P <= 0)
        return hipSuccess;
    int64_t blocks = (2 * P + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(adj_zero_acc, dim3((unsigned)blocks), dim3(256), 0, s, a.ws, 2 * P);
    return hipGetLastError();
}

template <typename T, int HK>
static hipError_t launch_bwd_t(const BwdArgs &a, int grid, hipStream_t s)
{
    const size_t shm = tile_shared_bytes((int)sizeof(Rec<T>), true);
    const hipError_t e = ensure_dynamic_lds(
        reinterpret_cast<const void *>(&pairwise_adjoint_tiles<T, HK>), (int)shm);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((pairwise_adjoint_tiles<T, HK>), dim3(grid), dim3(kThreads), shm, s, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_bwd_k(int hk, const BwdArgs &a, int grid, hipStream_t s)
{
    switch (hk) {
    case kAbs: return launch_bwd_t<T, kAbs>(a, grid, s);
    case kSqr: return launch_bwd_t<T, kSqr>(a, grid, s);
    case kProd: return launch_bwd_t<T, kProd>(a, grid, s);
    default: return launch_bwd_t<T, kPow>(a, grid, s);
    }
}

hipError_t launch_backward(int hk, bool f64, const BwdArgs &a, int grid, hipStream_t s)
{
    return f64 ? launch_bwd_k<double>(hk, a, grid, s) : launch_bwd_k<float>(hk, a, grid, s);
}

}  // namespace pcf
