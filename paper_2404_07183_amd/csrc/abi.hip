// abi.hip -- the C ABI declared in include/pcf.h: argument checks, host
// planning, workspace set-up and kernel launches.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <limits>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "launch.hpp"
#include "reduce.hpp"
#include "pcf.h"
#include "plan.hpp"


using namespace pcf;

namespace {

thread_local std::string g_err;

pcf_status fail(pcf_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

pcf_status hip_fail(hipError_t e, const char *what)
{
    return fail(PCF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int rec_bytes_of(pcf_dtype d) { return d == PCF_F64 ? 16 : 8; }

TileShape shape_of(uint32_t flags)
{
    TileShape s;
    const int32_t mb = (int32_t)((flags >> 8) & 63u);
    const int32_t bd = (int32_t)((flags >> 16) & 15u);
    if (mb >= 1 && mb <= kMaxBlock)
        s.max_block = mb;
    if (bd >= 2 && bd <= 8)
        s.budget_div = bd;
    return s;
}

constexpr int HK_ABS = kAbs, HK_SQR = kSqr, HK_PROD = kProd, HK_POW = kPow;

// The forward's h for an L_p kind: exact products for p = 1 and 2, squaring
// for other integer p (up to 64); in FP64 squaring plus one square root for
// p = k + 1/2 and the pow series otherwise; in FP32 the hardware base-2 log
// and exp for every non-integer p (faster there than the square root).
int lp_hkind(double p, bool f64)
{
    if (p == 1.0)
        return HK_ABS;
    if (p == 2.0)
        return HK_SQR;
    if (p <= 64.0 && floor(p) == p)
        return kPowInt;
    if (!f64)
        return HK_POW;
    if (p <= 64.0 && floor(2.0 * p) == 2.0 * p)
        return kPowHalf;
    return HK_POW;
}

int device_cus()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 256;
    static int cached[64] = {0};
    if (dev >= 0 && dev < 64 && cached[dev] > 0)
        return cached[dev];
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                              dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (dev >= 0 && dev < 64)
        cached[dev] = cus;
    return cus;
}

pcf_status check_set(const pcf_set *X)
{
    if (!X)
        return fail(PCF_EINVAL, "X is NULL");
    if (X->n < 0)
        return fail(PCF_EINVAL, "X->n < 0");
    if (X->dtype != PCF_F32 && X->dtype != PCF_F64)
        return fail(PCF_EINVAL, "X->dtype is not PCF_F32 or PCF_F64");
    if (X->n > 0 && (!X->offsets || !X->t || !X->v))
        return fail(PCF_EINVAL, "X has a NULL device pointer");
    return PCF_OK;
}

// Host copy of X->offsets (the caller's, or a synchronous device copy).
pcf_status host_offsets(const pcf_set *X, std::vector<int64_t> &buf,
                        const int64_t *&out, hipStream_t s)
{
    if (X->offsets_host) {
        out = X->offsets_host;
        return PCF_OK;
    }
    buf.resize((size_t)X->n + 1);
    hipError_t e = hipMemcpyAsync(buf.data(), X->offsets,
                                  sizeof(int64_t) * (size_t)(X->n + 1),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "copying offsets to the host");
    out = buf.data();
    return PCF_OK;
}

// What plan each workspace holds (the last one this library uploaded into
// it): the call it was made for, with everything that shapes its tiles and
// output mapping. A call with PCF_REUSE_PLAN is refused unless its workspace
// holds a plan made for that very call (same kind of call, record size,
// number of PCFs, window, leading dimension, upper-only and tile-shape
// flags; for a batched call the number of problems). The offsets' contents
// cannot be compared without reading them; the caller keeps them unchanged.
enum PlanKind { kPlanForward = 0, kPlanBackward = 1, kPlanBatched = 2, kPlanCross = 3 };
struct PlanTag {
    int kind = -1;
    int rec_bytes = 0;
    int64_t n = 0, r0 = 0, r1 = 0, c0 = 0, c1 = 0, ldo = 0;
    uint32_t shape_flags = 0;
    bool operator==(const PlanTag &o) const
    {
        return kind == o.kind && rec_bytes == o.rec_bytes && n == o.n && r0 == o.r0 &&
               r1 == o.r1 && c0 == o.c0 && c1 == o.c1 && ldo == o.ldo &&
               shape_flags == o.shape_flags;
    }
};
std::mutex g_plan_mu;
std::unordered_map<const void *, PlanTag> g_plan_tags;

PlanTag plan_tag(int kind, const pcf_set *X, const pcf_window *w, int64_t ldo, uint32_t flags)
{
    PlanTag t;
    t.kind = kind;
    t.rec_bytes = rec_bytes_of(X->dtype);
    t.n = X->n;
    if (w) {
        t.r0 = w->row0;
        t.r1 = w->row1;
        t.c0 = w->col0;
        t.c1 = w->col1;
    } else {
        t.r1 = t.c1 = -1;
    }
    t.ldo = ldo;
    t.shape_flags = flags & (PCF_UPPER_ONLY | 0x000fff00u);
    return t;
}

void remember_plan(const void *ws, const PlanTag &tag)
{
    std::lock_guard<std::mutex> lock(g_plan_mu);
    g_plan_tags[ws] = tag;
}

pcf_status check_reused_plan(const void *ws, const PlanTag &tag)
{
    std::lock_guard<std::mutex> lock(g_plan_mu);
    auto it = g_plan_tags.find(ws);
    if (it == g_plan_tags.end())
        return fail(PCF_EINVAL, "PCF_REUSE_PLAN: this workspace holds no plan made by "
                                "this library");
    const PlanTag &h = it->second;
    if (h.kind != tag.kind) {
        static const char *names[] = {"a matrix call", "pcf_pairwise_backward",
                                      "pcf_pairwise_batched", "pcf_cross"};
        return fail(PCF_EINVAL, std::string("PCF_REUSE_PLAN: the workspace holds a plan "
                                            "for ") + names[h.kind]);
    }
    if (h.rec_bytes != tag.rec_bytes)
        return fail(PCF_EINVAL, std::string("PCF_REUSE_PLAN: the workspace's plan was made "
                                            "for ") + (h.rec_bytes == 16 ? "FP64" : "FP32") +
                                    " data");
    if (!(h == tag))
        return fail(PCF_EINVAL, "PCF_REUSE_PLAN: the workspace's plan was made for another "
                                "set size, window, leading dimension or tile shape");
    return PCF_OK;
}

// Copy a plan's header, blocks and segments into the workspace.
pcf_status upload_plan(const Plan &plan, int rec_bytes, void *ws,
                       size_t ws_bytes, hipStream_t s, const PlanTag &tag)
{
    const int64_t need = plan_workspace_bytes(plan, rec_bytes);
    if ((int64_t)ws_bytes < need)
        return fail(PCF_ENOMEM, "workspace too small: need " +
                                    std::to_string(need) + " bytes, got " +
                                    std::to_string(ws_bytes));
    if (plan.rec_count >= ((int64_t)1 << 31))
        return fail(PCF_EUNSUPPORTED,
                    "more than 2^31 breakpoint records in one set");
    std::vector<unsigned char> buf;
    WsHeader hdr;
    plan_serialise(plan, rec_bytes, buf, hdr);
    hipError_t e = hipMemcpyAsync(ws, buf.data(), buf.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);  // buf is a local
    if (e != hipSuccess)
        return hip_fail(e, "uploading the tile plan");
    remember_plan(ws, tag);
    return PCF_OK;
}

pcf_status run_validation(const pcf_set *X, unsigned char *ws, int64_t P,
                          hipStream_t s, int64_t *first_bad)
{
    const int64_t init = std::numeric_limits<int64_t>::max();
    hipError_t e = hipMemcpyAsync(ws + offsetof(WsHeader, first_bad), &init,
                                  sizeof(init), hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return hip_fail(e, "validation set-up");
    e = X->dtype == PCF_F64
            ? launch_validate<double>(X->offsets, X->n, X->t, X->v, ws, P, s)
            : launch_validate<float>(X->offsets, X->n, X->t, X->v, ws, P, s);
    if (e != hipSuccess)
        return hip_fail(e, "validation launch");
    int64_t bad = init;
    e = hipMemcpyAsync(&bad, ws + offsetof(WsHeader, first_bad), sizeof(bad),
                       hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "validation read-back");
    *first_bad = (bad == init) ? -1 : bad;
    return PCF_OK;
}

struct Call {
    bool reuse;
    bool validate;
    int64_t P;  // rows, -1 when unknown (plan reused)
};

pcf_status prepare(const pcf_set *X, const Plan *plan, void *ws,
                   size_t ws_bytes, uint32_t flags, hipStream_t s, Call &c,
                   const int64_t *ho, const PlanTag &tag)
{
    c.reuse = (flags & PCF_REUSE_PLAN) != 0;
    c.validate = (flags & PCF_VALIDATE) != 0;
    c.P = ho ? ho[X->n] : -1;
    if (!c.reuse) {
        pcf_status st = upload_plan(*plan, rec_bytes_of(X->dtype), ws,
                                    ws_bytes, s, tag);
        if (st != PCF_OK)
            return st;
    } else {
        pcf_status st = check_reused_plan(ws, tag);
        if (st != PCF_OK)
            return st;
    }
    if (c.validate) {
        if (c.P < 0)
            return fail(PCF_EINVAL, "PCF_VALIDATE needs host offsets when "
                                    "the plan is reused");
        int64_t bad = -1;
        pcf_status st = run_validation(X, (unsigned char *)ws, c.P, s, &bad);
        if (st != PCF_OK)
            return st;
        if (bad >= 0)
            return fail(PCF_EDATA, "PCF " + std::to_string(bad) +
                                       " breaks the data contract (first "
                                       "time 0, strictly increasing finite "
                                       "times, finite values, last value 0)");
    }
    if ((flags & PCF_RECORDS_PACKED) && !c.reuse)
        return fail(PCF_EINVAL, "PCF_RECORDS_PACKED needs PCF_REUSE_PLAN");
    unsigned char *w = (unsigned char *)ws;
    hipError_t e = launch_reset(w, s);
    if (e == hipSuccess && !(flags & PCF_RECORDS_PACKED)) {
        // grid-stride; with an unknown row count use a full-chip grid
        const int64_t P = c.P >= 0 ? c.P : (int64_t)1 << 40;
        e = X->dtype == PCF_F64
                ? launch_pack<double>(X->offsets, X->n, X->t, X->v, w, P, s)
                : launch_pack<float>(X->offsets, X->n, X->t, X->v, w, P, s);
    }
    if (e != hipSuccess)
        return hip_fail(e, "packing breakpoint records");
    return PCF_OK;
}

int tile_grid(const Plan *plan, bool reuse)
{
    int grid = device_cus() * kWgPerCu;
    if (!reuse && plan && plan->ntiles < grid)
        grid = (int)(plan->ntiles > 0 ? plan->ntiles : 1);
    return grid;
}

pcf_status forward_common(const pcf_set *X, pcf_kind kind, double p, void *out,
                          int64_t ldo, const pcf_window *w, void *ws,
                          size_t ws_bytes, uint32_t flags, void *stream,
                          int accumulate = 0, double coef = 1.0)
{
    pcf_status st = check_set(X);
    if (st != PCF_OK)
        return st;
    if (kind != PCF_LP && kind != PCF_LP_POW && kind != PCF_GRAM)
        return fail(PCF_EINVAL, "unknown kind");
    if (kind != PCF_GRAM && (!(p >= 1.0) || !isfinite(p)))
        return fail(PCF_EINVAL, "p must be finite and >= 1");
    if (X->n == 0)
        return PCF_OK;
    if (!out || !ws)
        return fail(PCF_EINVAL, "out or ws is NULL");
    if (w && (w->row0 < 0 || w->row1 < w->row0 || w->row1 > X->n ||
              w->col0 < 0 || w->col1 < w->col0 || w->col1 > X->n))
        return fail(PCF_EINVAL, "window out of range");
    const int64_t width = w ? (w->col1 - w->col0) : X->n;
    if (ldo < width || ldo < 1)
        return fail(PCF_EINVAL, "ldo smaller than the output width");
    if (w && (w->row1 == w->row0 || w->col1 == w->col0))
        return PCF_OK;
    hipStream_t s = (hipStream_t)stream;
    const bool reuse = (flags & PCF_REUSE_PLAN) != 0;

    Plan plan;
    std::vector<int64_t> obuf;
    const int64_t *ho = X->offsets_host;
    if (!reuse) {
        st = host_offsets(X, obuf, ho, s);
        if (st != PCF_OK)
            return st;
        std::string err;
        if (!plan_matrix(X->n, ho, rec_bytes_of(X->dtype), false, w != nullptr,
                         w ? w->row0 : 0, w ? w->row1 : 0, w ? w->col0 : 0,
                         w ? w->col1 : 0, (flags & PCF_UPPER_ONLY) != 0, ldo,
                         shape_of(flags), plan, err))
            return fail(PCF_EINVAL, err);
    }
    Call c;
    st = prepare(X, reuse ? nullptr : &plan, ws, ws_bytes, flags, s, c, ho,
                 plan_tag(kPlanForward, X, w, ldo, flags));
    if (st != PCF_OK)
        return st;

    FwdArgs a;
    a.offsets = X->offsets;
    a.ws = (unsigned char *)ws;
    a.out = out;
    a.p = p;
    a.inv_p = 1.0 / p;
    a.gram = kind == PCF_GRAM ? 1 : 0;
    a.accumulate = accumulate;
    a.coef = coef;
    int hk;
    if (kind == PCF_GRAM) {
        hk = HK_PROD;
        a.root = 0;
    } else {
        hk = lp_hkind(p, X->dtype == PCF_F64);
        a.root = (kind == PCF_LP_POW || p == 1.0) ? 0 : (p == 2.0 ? 1 : 2);
    }
    if (accumulate && a.root != 0)
        return fail(PCF_EINVAL, "a term of a sum takes no root");
    hipError_t e = launch_forward(X->dtype == PCF_F64, hk, a,
                                  tile_grid(reuse ? nullptr : &plan, reuse), s);
    if (e != hipSuccess)
        return hip_fail(e, "tile kernel launch");
    return PCF_OK;
}

// The combined CSR of X then Y (host), and the plan of the window
// [0, nx) x [nx, nx + ny) over it.
pcf_status cross_plan(const pcf_set *X, const pcf_set *Y, int64_t ldo, uint32_t flags,
                      hipStream_t s, std::vector<int64_t> &comb, Plan &plan)
{
    std::vector<int64_t> xb, yb;
    const int64_t *xo = X->offsets_host, *yo = Y->offsets_host;
    pcf_status st = host_offsets(X, xb, xo, s);
    if (st == PCF_OK)
        st = host_offsets(Y, yb, yo, s);
    if (st != PCF_OK)
        return st;
    const int64_t nx = X->n, ny = Y->n;
    comb.resize((size_t)(nx + ny + 1));
    for (int64_t i = 0; i <= nx; ++i)
        comb[i] = xo[i];
    for (int64_t i = 1; i <= ny; ++i)
        comb[nx + i] = xo[nx] + yo[i];
    std::string err;
    if (!plan_matrix(nx + ny, comb.data(), rec_bytes_of(X->dtype), false, true, 0, nx,
                     nx, nx + ny, false, ldo, shape_of(flags), plan, err))
        return fail(PCF_EINVAL, err);
    return PCF_OK;
}

// Bytes of the cross-set workspace: the plan's, then the combined device
// offsets.
int64_t cross_offsets_at(const Plan &plan, int rec_bytes, bool bound)
{
    return bound ? plan_workspace_bound(plan, rec_bytes)
                 : plan_workspace_bytes(plan, rec_bytes);
}

pcf_status check_pair(const pcf_set *X, const pcf_set *Y)
{
    pcf_status st = check_set(X);
    if (st == PCF_OK)
        st = check_set(Y);
    if (st != PCF_OK)
        return st;
    if (X->dtype != Y->dtype)
        return fail(PCF_EINVAL, "X and Y have different dtypes");
    return PCF_OK;
}

// offsets_out[1..n] hold per-PCF row counts written by a count kernel on
// s (-1: a PCF the transform cannot carry): copy them to the host, turn
// them into offsets there and copy those back. Synchronous, as the caller
// needs the total to allocate the rows.
pcf_status counts_to_offsets(int64_t n, int64_t *offsets_out, int64_t *offsets_out_host,
                             hipStream_t s, const char *what)
{
    hipError_t e = hipSuccess;
    if (n == 0)
        offsets_out_host[0] = 0;
    else
        e = hipMemcpyAsync(offsets_out_host, offsets_out, sizeof(int64_t) * (size_t)(n + 1),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "reading the row counts");
    for (int64_t i = 0; i < n; ++i) {
        if (offsets_out_host[i + 1] < 0)
            return fail(PCF_EINVAL, std::string("PCF ") + std::to_string(i) +
                                        ": its " + what + " times are not finite and increasing");
        offsets_out_host[i + 1] += offsets_out_host[i];
    }
    e = hipMemcpyAsync(offsets_out, offsets_out_host, sizeof(int64_t) * (size_t)(n + 1),
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);  // offsets_out_host may be a local
    return e == hipSuccess ? PCF_OK : hip_fail(e, "writing the offsets");
}

// A time weight: exponential needs 0 < c < inf, power -1 < c < inf.
pcf_status check_weight(int weight, double c)
{
    if (weight == PCF_WEIGHT_EXP && c > 0.0 && isfinite(c))
        return PCF_OK;
    if (weight == PCF_WEIGHT_POW && c > -1.0 && isfinite(c))
        return PCF_OK;
    return fail(PCF_EINVAL, "weight: PCF_WEIGHT_EXP needs c > 0, PCF_WEIGHT_POW c > -1");
}

// A reduction's host plan: group checks, the tree depth and the workspace
// layout (group offsets and the root pass's chunk table, chunk counts and
// output offsets, two ping-pong row buffers, the deviation sums of a
// standard deviation).
constexpr int64_t kRedChunkRows = 1024;  // the root pass's chunk (reduce.hip)
constexpr int64_t kRedStdSlots = 64;     // the std pass's bounds per chunk (reduce.hip)

struct RedPlan {
    int32_t B = 0;
    int L = 0;
    int64_t n = 0, P = 0, C = 0;  // PCFs, rows, chunks
    std::vector<int64_t> meta;    // groups (B+1), chunk rows (C), chunk groups (C)
    size_t off_ccnt = 0, off_coff = 0, off_buf[4] = {0, 0, 0, 0}, off_q = 0, off_map = 0;
    size_t off_kb = 0;  // PCF_REDUCE_STD: each chunk's first rows (64 per chunk)
    size_t bytes = 0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

pcf_status red_plan(const pcf_set *X, int32_t B, const int64_t *groups, int op,
                    hipStream_t s, RedPlan &rp)
{
    pcf_status st = check_set(X);
    if (st != PCF_OK)
        return st;
    if (op < RO_SUM || op > RO_SQDIFF)
        return fail(PCF_EINVAL, "unknown reduction op");
    if (B < 0 || (B > 0 && !groups))
        return fail(PCF_EINVAL, "B < 0 or group_offsets_host is NULL");
    const int64_t n = X->n;
    if (B == 0 ? n != 0 : (groups[0] != 0 || groups[B] != n))
        return fail(PCF_EINVAL, "the groups must cover the set's PCFs 0 .. n-1");
    if (n >= ((int64_t)1 << 31))
        return fail(PCF_EUNSUPPORTED, "reductions take fewer than 2^31 PCFs");
    int64_t mmax = 0;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t m = groups[b + 1] - groups[b];
        if (m < (op == PCF_REDUCE_STD ? 2 : 1))
            return fail(PCF_EINVAL, "group " + std::to_string(b) + " has " + std::to_string(m) +
                                        " PCFs (at least 1, 2 for PCF_REDUCE_STD)");
        if (op == PCF_REDUCE_STD && m >= ((int64_t)1 << 30))
            return fail(PCF_EUNSUPPORTED, "a standard deviation over 2^30 or more PCFs");
        mmax = m > mmax ? m : mmax;
    }
    std::vector<int64_t> obuf;
    const int64_t *ho = nullptr;
    if (n > 0) {
        st = host_offsets(X, obuf, ho, s);
        if (st != PCF_OK)
            return st;
        for (int64_t i = 0; i < n; ++i)
            if (ho[i + 1] <= ho[i])
                return fail(PCF_EINVAL, "PCF " + std::to_string(i) + " has no rows");
    }
    rp.B = B;
    rp.n = n;
    rp.P = n > 0 ? ho[n] : 0;
    rp.L = 0;
    while (((int64_t)1 << rp.L) < mmax)
        ++rp.L;
    if (groups)
        rp.meta.assign(groups, groups + B + 1);
    else
        rp.meta.assign(1, 0);
    std::vector<int64_t> crow, cgrp;
    for (int32_t b = 0; b < B; ++b)
        for (int64_t r = ho[groups[b]]; r < ho[groups[b + 1]]; r += kRedChunkRows) {
            crow.push_back(r);
            cgrp.push_back(b);
        }
    rp.C = (int64_t)crow.size();
    rp.meta.insert(rp.meta.end(), crow.begin(), crow.end());
    rp.meta.insert(rp.meta.end(), cgrp.begin(), cgrp.end());
    const size_t esz = X->dtype == PCF_F64 ? 8 : 4;
    const size_t cbytes = align256((size_t)(rp.C > 0 ? rp.C : 1) * sizeof(int64_t));
    size_t off = align256(rp.meta.size() * sizeof(int64_t));
    rp.off_ccnt = off;
    off += cbytes;
    rp.off_coff = off;
    off += cbytes;
    for (int k = 0; k < 4; ++k) {
        rp.off_buf[k] = off;
        off += align256((size_t)(rp.P > 0 ? rp.P : 1) * esz);
    }
    rp.off_q = off;
    off += align256((size_t)(rp.P > 0 ? rp.P : 1) * esz);
    rp.off_map = off;
    off += align256((size_t)(rp.P > 0 ? rp.P : 1) * sizeof(int32_t));
    if (op == PCF_REDUCE_STD) {
        rp.off_kb = off;
        off += align256((size_t)(rp.C > 0 ? rp.C : 1) * kRedStdSlots * sizeof(int64_t));
    }
    rp.bytes = off;
    return PCF_OK;
}

// The bounds of a restriction in the set's precision: 0 <= a < b <= inf,
// both still ordered (and b still finite when given finite) once rounded.
pcf_status check_range(const pcf_set *X, double a, double b)
{
    if (!(a >= 0.0) || !isfinite(a) || !(b > a))
        return fail(PCF_EINVAL, "the bounds must satisfy 0 <= a < b (b may be inf)");
    if (X->dtype == PCF_F32) {
        const float fa = (float)a, fb = (float)b;
        if (!(fb > fa) || (isfinite(b) && !isfinite(fb)))
            return fail(PCF_EINVAL, "the bounds are not ordered once rounded to FP32");
    }
    return PCF_OK;
}

}  // namespace

namespace pcf {

// Used by noalloc.hip (the allocation-free entry point).
pcf_status noalloc_fail(pcf_status s, const std::string &msg) { return fail(s, msg); }

pcf_status noalloc_forward(const pcf_set *X, pcf_kind kind, double p, void *out,
                           int64_t ldo, const pcf_window *w, void *ws,
                           size_t ws_bytes, uint32_t flags, void *stream)
{
    return forward_common(X, kind, p, out, ldo, w, ws, ws_bytes, flags, stream);
}

// Exact workspace of a forward call's plan (the size forward_common uploads
// and packs), without touching a device when X->offsets_host is given.
pcf_status noalloc_plan_bytes(const pcf_set *X, const pcf_window *w, int64_t ldo,
                              uint32_t flags, int64_t *bytes)
{
    pcf_status st = check_set(X);
    if (st != PCF_OK)
        return st;
    if (w && (w->row0 < 0 || w->row1 < w->row0 || w->row1 > X->n || w->col0 < 0 ||
              w->col1 < w->col0 || w->col1 > X->n))
        return fail(PCF_EINVAL, "window out of range");
    std::vector<int64_t> obuf;
    const int64_t *ho = nullptr;
    st = host_offsets(X, obuf, ho, nullptr);
    if (st != PCF_OK)
        return st;
    Plan plan;
    std::string err;
    if (!plan_matrix(X->n, ho, rec_bytes_of(X->dtype), false, w != nullptr,
                     w ? w->row0 : 0, w ? w->row1 : 0, w ? w->col0 : 0, w ? w->col1 : 0,
                     (flags & PCF_UPPER_ONLY) != 0, ldo > 0 ? ldo : 1, shape_of(flags), plan,
                     err))
        return fail(PCF_EINVAL, err);
    *bytes = plan_workspace_bytes(plan, rec_bytes_of(X->dtype));
    return PCF_OK;
}

// Workspace of a sum of terms: the forward's (planned on X; a warped set has
// no more rows), then the warped set's offsets, times and values.
struct TermsLayout {
    size_t fwd = 0, off = 0, t = 0, v = 0, bytes = 0;
};

pcf_status terms_layout(const pcf_set *X, const pcf_window *w, uint32_t flags,
                        TermsLayout &L)
{
    int64_t fb = 0;
    const int64_t ldo = w ? (w->col1 - w->col0) : X->n;
    pcf_status st = noalloc_plan_bytes(X, w, ldo, flags & ~(uint32_t)PCF_UPPER_ONLY, &fb);
    if (st != PCF_OK)
        return st;
    std::vector<int64_t> obuf;
    const int64_t *ho = nullptr;
    st = host_offsets(X, obuf, ho, nullptr);
    if (st != PCF_OK)
        return st;
    const size_t rows = X->n > 0 ? (size_t)ho[X->n] : 0;
    const size_t esz = X->dtype == PCF_F64 ? 8 : 4;
    L.fwd = align256((size_t)fb);
    L.off = L.fwd;
    L.t = L.off + align256((size_t)(X->n + 1) * sizeof(int64_t));
    L.v = L.t + align256((rows > 0 ? rows : 1) * esz);
    L.bytes = L.v + align256((rows > 0 ? rows : 1) * esz);
    return PCF_OK;
}

pcf_status check_terms(int32_t nterms, const pcf_term *terms, double q)
{
    if (nterms < 1 || !terms)
        return fail(PCF_EINVAL, "at least one term is needed");
    for (int32_t m = 0; m < nterms; ++m) {
        const pcf_term &T = terms[m];
        const std::string who = "term " + std::to_string(m) + ": ";
        if (T.kind != PCF_LP_POW && T.kind != PCF_GRAM)
            return fail(PCF_EINVAL, who + "kind must be PCF_LP_POW or PCF_GRAM");
        if (T.kind == PCF_LP_POW && (!(T.p >= 1.0) || !isfinite(T.p)))
            return fail(PCF_EINVAL, who + "p must be finite and >= 1");
        if (T.weight != 0 && check_weight(T.weight, T.c) != PCF_OK)
            return fail(PCF_EINVAL, who + "bad weight");
        if (!isfinite(T.coef))
            return fail(PCF_EINVAL, who + "the coefficient is not finite");
    }
    if (!(q == 0.0 || (q >= 1.0 && isfinite(q))))
        return fail(PCF_EINVAL, "the root q must be 0 (none) or finite and >= 1");
    return PCF_OK;
}

}  // namespace pcf

extern "C" {

pcf_status pcf_terms_workspace_bytes(const pcf_set *X, const pcf_window *w, uint32_t flags,
                                     size_t *bytes)
{
    if (!bytes)
        return fail(PCF_EINVAL, "bytes is NULL");
    TermsLayout L;
    pcf_status st = terms_layout(X, w, flags, L);
    if (st != PCF_OK)
        return st;
    *bytes = L.bytes;
    return PCF_OK;
}

pcf_status pcf_pairwise_terms(const pcf_set *X, int32_t nterms, const pcf_term *terms,
                              double q, void *out, int64_t ldo, const pcf_window *w,
                              void *ws, size_t ws_bytes, uint32_t flags, void *stream)
{
    pcf_status st = check_set(X);
    if (st == PCF_OK)
        st = check_terms(nterms, terms, q);
    if (st != PCF_OK)
        return st;
    if (flags & (PCF_REUSE_PLAN | PCF_RECORDS_PACKED))
        return fail(PCF_EINVAL, "every term plans and packs its own set: no plan reuse");
    if (X->n == 0)
        return PCF_OK;
    if (!out || !ws)
        return fail(PCF_EINVAL, "out or ws is NULL");
    TermsLayout L;
    st = terms_layout(X, w, flags, L);
    if (st != PCF_OK)
        return st;
    if (ws_bytes < L.bytes)
        return fail(PCF_ENOMEM, "workspace too small: need " + std::to_string(L.bytes) +
                                    " bytes (pcf_terms_workspace_bytes)");
    hipStream_t s = (hipStream_t)stream;
    unsigned char *wb = (unsigned char *)ws;
    std::vector<int64_t> zoff((size_t)X->n + 1);
    for (int32_t m = 0; m < nterms; ++m) {
        const pcf_term &T = terms[m];
        pcf_set Z = *X;
        if (T.weight != 0) {
            // the set warped by this term's weight, in the workspace
            int64_t *off = (int64_t *)(wb + L.off);
            hipError_t e = launch_warp_count(X->dtype == PCF_F64, X->offsets, X->n, X->t,
                                             (int)T.weight, T.c, off, s);
            if (e != hipSuccess)
                return hip_fail(e, "warp count launch");
            st = counts_to_offsets(X->n, off, zoff.data(), s, "warped");
            if (st != PCF_OK)
                return st;
            e = launch_warp_fill(X->dtype == PCF_F64, X->offsets, X->n, X->t, X->v,
                                 (int)T.weight, T.c, off, wb + L.t, wb + L.v, s);
            if (e != hipSuccess)
                return hip_fail(e, "warp kernel launch");
            Z.offsets = off;
            Z.t = wb + L.t;
            Z.v = wb + L.v;
            Z.offsets_host = zoff.data();
        }
        st = forward_common(&Z, T.kind, T.kind == PCF_GRAM ? 0.0 : T.p, out, ldo, w, ws,
                            L.fwd, flags & ~(uint32_t)PCF_DETERMINISTIC, stream,
                            m == 0 ? 2 : 1, T.coef);
        if (st != PCF_OK)
            return st;
        // (the next term's warp rewrites the area after this term's kernels
        // on the same stream)
    }
    if (q > 1.0) {
        const int64_t rows = w ? w->row1 - w->row0 : X->n, cols = w ? w->col1 - w->col0 : X->n;
        hipError_t e = launch_apply_root(X->dtype == PCF_F64, out, rows, cols, ldo, q,
                                         (flags & PCF_UPPER_ONLY) != 0, w ? w->row0 : 0,
                                         w ? w->col0 : 0, s);
        if (e != hipSuccess)
            return hip_fail(e, "root launch");
    }
    return PCF_OK;
}

const char *pcf_last_error(void) { return g_err.c_str(); }

int pcf_abi_version(void) { return 1; }

pcf_status pcf_workspace_bytes(const pcf_set *X, pcf_kind kind,
                               const pcf_window *w, int backward,
                               size_t *bytes)
{
    (void)kind;
    pcf_status st = check_set(X);
    if (st != PCF_OK)
        return st;
    if (!bytes)
        return fail(PCF_EINVAL, "bytes is NULL");
    if (X->n == 0) {
        *bytes = (size_t)kHeaderBytes;
        return PCF_OK;
    }
    std::vector<int64_t> obuf;
    const int64_t *ho = nullptr;
    st = host_offsets(X, obuf, ho, nullptr);
    if (st != PCF_OK)
        return st;
    Plan plan;
    std::string err;
    const int64_t ldo = w ? (w->col1 - w->col0) : X->n;
    if (!plan_matrix(X->n, ho, rec_bytes_of(X->dtype), backward != 0,
                     w != nullptr, w ? w->row0 : 0, w ? w->row1 : 0,
                     w ? w->col0 : 0, w ? w->col1 : 0, false,
                     ldo > 0 ? ldo : 1, TileShape(), plan, err))
        return fail(PCF_EINVAL, err);
    *bytes = (size_t)plan_workspace_bound(plan, rec_bytes_of(X->dtype));
    return PCF_OK;
}

pcf_status pcf_pairwise_lp(const pcf_set *X, pcf_kind kind, double p,
                           void *out, int64_t ldo, const pcf_window *w,
                           void *ws, size_t ws_bytes, uint32_t flags,
                           void *stream)
{
    if (kind != PCF_LP && kind != PCF_LP_POW)
        return fail(PCF_EINVAL, "pcf_pairwise_lp takes PCF_LP or PCF_LP_POW");
    return forward_common(X, kind, p, out, ldo, w, ws, ws_bytes, flags,
                          stream);
}

pcf_status pcf_gram(const pcf_set *X, void *out, int64_t ldo,
                    const pcf_window *w, void *ws, size_t ws_bytes,
                    uint32_t flags, void *stream)
{
    return forward_common(X, PCF_GRAM, 0.0, out, ldo, w, ws, ws_bytes, flags,
                          stream);
}

pcf_status pcf_batched_workspace_bytes(int32_t B,
                                       const int64_t *set_offsets_host,
                                       const pcf_set *all, size_t *bytes)
{
    pcf_status st = check_set(all);
    if (st != PCF_OK)
        return st;
    if (!bytes)
        return fail(PCF_EINVAL, "bytes is NULL");
    std::vector<int64_t> obuf;
    const int64_t *ho = nullptr;
    if (all->n > 0) {
        st = host_offsets(all, obuf, ho, nullptr);
        if (st != PCF_OK)
            return st;
    }
    std::vector<int64_t> oo((size_t)(B > 0 ? B : 0), 0);
    Plan plan;
    std::string err;
    if (!plan_batched(B, set_offsets_host, oo.data(), ho, all->n,
                      rec_bytes_of(all->dtype), false, TileShape(), plan, err))
        return fail(PCF_EINVAL, err);
    *bytes = (size_t)plan_workspace_bound(plan, rec_bytes_of(all->dtype));
    return PCF_OK;
}

pcf_status pcf_pairwise_batched(int32_t B, const int64_t *set_offsets_host,
                                const pcf_set *all, pcf_kind kind, double p,
                                void *out, const int64_t *out_offsets_host,
                                void *ws, size_t ws_bytes, uint32_t flags,
                                void *stream)
{
    pcf_status st = check_set(all);
    if (st != PCF_OK)
        return st;
    if (kind != PCF_LP && kind != PCF_LP_POW && kind != PCF_GRAM)
        return fail(PCF_EINVAL, "unknown kind");
    if (kind != PCF_GRAM && (!(p >= 1.0) || !isfinite(p)))
        return fail(PCF_EINVAL, "p must be finite and >= 1");
    if (B < 0)
        return fail(PCF_EINVAL, "B < 0");
    if (B == 0 || all->n == 0)
        return PCF_OK;
    if (!out || !ws)
        return fail(PCF_EINVAL, "out or ws is NULL");
    hipStream_t s = (hipStream_t)stream;
    const bool reuse = (flags & PCF_REUSE_PLAN) != 0;
    Plan plan;
    std::vector<int64_t> obuf;
    const int64_t *ho = all->offsets_host;
    if (!reuse) {
        if (!set_offsets_host || !out_offsets_host)
            return fail(PCF_EINVAL, "set_offsets_host or out_offsets_host is NULL");
        st = host_offsets(all, obuf, ho, s);
        if (st != PCF_OK)
            return st;
        std::string err;
        if (!plan_batched(B, set_offsets_host, out_offsets_host, ho, all->n,
                          rec_bytes_of(all->dtype),
                          (flags & PCF_UPPER_ONLY) != 0, shape_of(flags), plan,
                          err))
            return fail(PCF_EINVAL, err);
    }
    Call c;
    {
        PlanTag tag = plan_tag(kPlanBatched, all, nullptr, 0, flags);
        tag.ldo = B;
        st = prepare(all, reuse ? nullptr : &plan, ws, ws_bytes, flags, s, c, ho, tag);
    }
    if (st != PCF_OK)
        return st;
    FwdArgs a;
    a.offsets = all->offsets;
    a.ws = (unsigned char *)ws;
    a.out = out;
    a.p = p;
    a.inv_p = 1.0 / p;
    a.gram = kind == PCF_GRAM ? 1 : 0;
    int hk;
    if (kind == PCF_GRAM) {
        hk = HK_PROD;
        a.root = 0;
    } else {
        hk = lp_hkind(p, all->dtype == PCF_F64);
        a.root = (kind == PCF_LP_POW || p == 1.0) ? 0 : (p == 2.0 ? 1 : 2);
    }
    hipError_t e = launch_forward(all->dtype == PCF_F64, hk, a,
                                  tile_grid(reuse ? nullptr : &plan, reuse), s);
    if (e != hipSuccess)
        return hip_fail(e, "tile kernel launch");
    return PCF_OK;
}

pcf_status pcf_validate(const pcf_set *X, int64_t *first_bad, void *ws,
                        size_t ws_bytes, void *stream)
{
    pcf_status st = check_set(X);
    if (st != PCF_OK)
        return st;
    if (!first_bad)
        return fail(PCF_EINVAL, "first_bad is NULL");
    if (!ws || ws_bytes < (size_t)kHeaderBytes)
        return fail(PCF_ENOMEM, "validation needs 256 bytes of workspace");
    *first_bad = -1;
    if (X->n == 0)
        return PCF_OK;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> obuf;
    const int64_t *ho = nullptr;
    st = host_offsets(X, obuf, ho, s);
    if (st != PCF_OK)
        return st;
    for (int64_t i = 0; i < X->n; ++i) {
        if (ho[i + 1] <= ho[i]) {
            *first_bad = i;
            return PCF_OK;
        }
    }
    return run_validation(X, (unsigned char *)ws, ho[X->n], s, first_bad);
}

pcf_status pcf_plan_inspect(int64_t n, const int64_t *offsets_host,
                            pcf_dtype dtype, const pcf_window *w,
                            int backward, int64_t *nblocks, int64_t *nseg,
                            int64_t *ntiles, int32_t *blocks_out,
                            int64_t blocks_cap)
{
    if (dtype != PCF_F32 && dtype != PCF_F64)
        return fail(PCF_EINVAL, "bad dtype");
    Plan plan;
    std::string err;
    const int64_t ldo = w ? (w->col1 - w->col0) : n;
    if (!plan_matrix(n, offsets_host, rec_bytes_of(dtype), backward != 0,
                     w != nullptr, w ? w->row0 : 0, w ? w->row1 : 0,
                     w ? w->col0 : 0, w ? w->col1 : 0, false,
                     ldo > 0 ? ldo : 1, TileShape(), plan, err))
        return fail(PCF_EINVAL, err);
    const int64_t nb = plan.blocks.empty() ? 0 : (int64_t)plan.blocks.size() - 1;
    if (nblocks)
        *nblocks = nb;
    if (nseg)
        *nseg = (int64_t)plan.segs.size();
    if (ntiles)
        *ntiles = plan.ntiles;
    if (blocks_out)
        for (int64_t i = 0; i < (int64_t)plan.blocks.size() && i < blocks_cap; ++i)
            blocks_out[i] = plan.blocks[i];
    return PCF_OK;
}

pcf_status pcf_pairwise_backward(const pcf_set *X, pcf_kind kind, double p,
                                 const void *grad_out, int64_t ldg,
                                 const void *fwd_out, int64_t ldf,
                                 void *grad_t, void *grad_v, void *ws,
                                 size_t ws_bytes, uint32_t flags,
                                 void *stream)
{
    pcf_status st = check_set(X);
    if (st != PCF_OK)
        return st;
    if (kind != PCF_LP && kind != PCF_LP_POW && kind != PCF_GRAM)
        return fail(PCF_EINVAL, "unknown kind");
    if (kind != PCF_GRAM && (!(p >= 1.0) || !isfinite(p)))
        return fail(PCF_EINVAL, "p must be finite and >= 1");
    const bool f64 = X->dtype == PCF_F64;
    const bool fixed = (flags & PCF_DETERMINISTIC) != 0;
    if (X->n == 0)
        return PCF_OK;
    const bool chain = kind == PCF_LP && p != 1.0;
    if (fixed && (X->n + 31) / 32 > 65535)
        return fail(PCF_EUNSUPPORTED, "PCF_DETERMINISTIC takes at most 2,097,120 PCFs");
    if (!grad_out || !grad_t || !grad_v || !ws)
        return fail(PCF_EINVAL, "grad_out, grad_t, grad_v or ws is NULL");
    if (chain && !fwd_out)
        return fail(PCF_EINVAL, "PCF_LP with p != 1 needs the forward result");
    if (ldg < X->n || (chain && ldf < X->n))
        return fail(PCF_EINVAL, "leading dimension smaller than n");
    hipStream_t s = (hipStream_t)stream;
    const bool reuse = (flags & PCF_REUSE_PLAN) != 0;
    Plan plan;
    std::vector<int64_t> obuf;
    const int64_t *ho = X->offsets_host;
    if (!reuse) {
        st = host_offsets(X, obuf, ho, s);
        if (st != PCF_OK)
            return st;
        std::string err;
        if (!plan_matrix(X->n, ho, rec_bytes_of(X->dtype), true, false, 0, 0,
                         0, 0, false, X->n, shape_of(flags), plan, err))
            return fail(PCF_EINVAL, err);
    }
    Call c;
    st = prepare(X, reuse ? nullptr : &plan, ws, ws_bytes, flags, s, c, ho,
                 plan_tag(kPlanBackward, X, nullptr, X->n, flags));
    if (st != PCF_OK)
        return st;
    const int64_t P = ho ? ho[X->n] : -1;
    if (P < 0)
        return fail(PCF_EINVAL, "the adjoint needs host offsets");
    hipError_t e = f64 ? launch_zero((double *)grad_t, P, s)
                       : launch_zero_f32((float *)grad_t, P, s);
    if (e == hipSuccess)
        e = f64 ? launch_zero((double *)grad_v, P, s) : launch_zero_f32((float *)grad_v, P, s);
    if (e != hipSuccess)
        return hip_fail(e, "clearing the gradients");
    BwdArgs a;
    a.offsets = X->offsets;
    a.ws = (unsigned char *)ws;
    a.grad_out = (const double *)grad_out;
    a.ldg = ldg;
    a.fwd_out = (const double *)fwd_out;
    a.ldf = ldf;
    a.grad_t = grad_t;
    a.grad_v = grad_v;
    a.p = p;
    a.chain = chain ? 1 : 0;
    a.gram = kind == PCF_GRAM ? 1 : 0;
    a.n = X->n;
    a.fixed = fixed ? 1 : 0;
    const int hk = kind == PCF_GRAM ? HK_PROD
                                    : (p == 1.0 ? HK_ABS : (p == 2.0 ? HK_SQR : HK_POW));
    if (fixed) {
        e = launch_adj_bounds(f64, a, s);
        if (e == hipSuccess && !f64)
            e = launch_adj_acc(a, P, s);
        if (e != hipSuccess)
            return hip_fail(e, "adjoint bounds launch");
    }
    e = launch_backward(hk, f64, a, tile_grid(reuse ? nullptr : &plan, reuse), s);
    if (e != hipSuccess)
        return hip_fail(e, "adjoint kernel launch");
    if (fixed) {
        e = launch_adj_finish(hk, f64, a, P, s);
        if (e != hipSuccess)
            return hip_fail(e, "adjoint finish launch");
    }
    return PCF_OK;
}

pcf_status pcf_cross_workspace_bytes(const pcf_set *X, const pcf_set *Y,
                                     size_t *bytes)
{
    pcf_status st = check_pair(X, Y);
    if (st != PCF_OK)
        return st;
    if (!bytes)
        return fail(PCF_EINVAL, "bytes is NULL");
    if (X->n == 0 || Y->n == 0) {
        *bytes = (size_t)kHeaderBytes;
        return PCF_OK;
    }
    std::vector<int64_t> comb;
    Plan plan;
    st = cross_plan(X, Y, Y->n, 0, nullptr, comb, plan);
    if (st != PCF_OK)
        return st;
    *bytes = (size_t)(cross_offsets_at(plan, rec_bytes_of(X->dtype), true) +
                      align_up((X->n + Y->n + 1) * 8, 256));
    return PCF_OK;
}

pcf_status pcf_cross(const pcf_set *X, const pcf_set *Y, pcf_kind kind, double p,
                     void *out, int64_t ldo, void *ws, size_t ws_bytes,
                     uint32_t flags, void *stream)
{
    pcf_status st = check_pair(X, Y);
    if (st != PCF_OK)
        return st;
    if (kind != PCF_LP && kind != PCF_LP_POW && kind != PCF_GRAM)
        return fail(PCF_EINVAL, "unknown kind");
    if (kind != PCF_GRAM && (!(p >= 1.0) || !isfinite(p)))
        return fail(PCF_EINVAL, "p must be finite and >= 1");
    if (flags & (PCF_UPPER_ONLY | PCF_REUSE_PLAN | PCF_RECORDS_PACKED))
        return fail(PCF_EINVAL, "pcf_cross takes neither PCF_UPPER_ONLY nor "
                                "PCF_REUSE_PLAN nor PCF_RECORDS_PACKED");
    if (X->n == 0 || Y->n == 0)
        return PCF_OK;
    if (!out || !ws)
        return fail(PCF_EINVAL, "out or ws is NULL");
    if (ldo < Y->n)
        return fail(PCF_EINVAL, "ldo smaller than Y->n");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> comb;
    Plan plan;
    st = cross_plan(X, Y, ldo, flags, s, comb, plan);
    if (st != PCF_OK)
        return st;
    const int rb = rec_bytes_of(X->dtype);
    const int64_t at = cross_offsets_at(plan, rb, false);
    const int64_t need = at + align_up((X->n + Y->n + 1) * 8, 256);
    if ((int64_t)ws_bytes < need)
        return fail(PCF_ENOMEM, "workspace too small: need " + std::to_string(need) +
                                    " bytes, got " + std::to_string(ws_bytes));
    st = upload_plan(plan, rb, ws, ws_bytes, s, plan_tag(kPlanCross, X, nullptr, ldo, flags));
    if (st != PCF_OK)
        return st;
    unsigned char *w = (unsigned char *)ws;
    if (flags & PCF_VALIDATE) {
        const pcf_set *sets[2] = {X, Y};
        for (int q = 0; q < 2; ++q) {
            int64_t bad = -1;
            const int64_t P = comb[q == 0 ? X->n : X->n + Y->n] - (q == 0 ? 0 : comb[X->n]);
            st = run_validation(sets[q], w, P, s, &bad);
            if (st != PCF_OK)
                return st;
            if (bad >= 0)
                return fail(PCF_EDATA, std::string(q == 0 ? "X" : "Y") + " PCF " +
                                           std::to_string(bad) +
                                           " breaks the data contract (first time "
                                           "0, strictly increasing finite times, "
                                           "finite values, last value 0)");
        }
    }
    // one record array: X's records, then Y's (starting past X's records and
    // padding), indexed through the combined offsets
    int64_t *coff = reinterpret_cast<int64_t *>(w + at);
    const int64_t px = comb[X->n], py = comb[X->n + Y->n] - px;
    const int64_t ybase = px + X->n * kPad;
    hipError_t e = launch_reset(w, s);
    if (e == hipSuccess)
        e = launch_concat_offsets(X->offsets, X->n, Y->offsets, Y->n, coff, s);
    if (e == hipSuccess)
        e = X->dtype == PCF_F64
                ? launch_pack<double>(X->offsets, X->n, X->t, X->v, w, px, s, 0)
                : launch_pack<float>(X->offsets, X->n, X->t, X->v, w, px, s, 0);
    if (e == hipSuccess)
        e = X->dtype == PCF_F64
                ? launch_pack<double>(Y->offsets, Y->n, Y->t, Y->v, w, py, s, ybase)
                : launch_pack<float>(Y->offsets, Y->n, Y->t, Y->v, w, py, s, ybase);
    if (e != hipSuccess)
        return hip_fail(e, "packing breakpoint records");

    FwdArgs a;
    a.offsets = coff;
    a.ws = w;
    a.out = out;
    a.p = p;
    a.inv_p = 1.0 / p;
    a.gram = kind == PCF_GRAM ? 1 : 0;
    int hk;
    if (kind == PCF_GRAM) {
        hk = HK_PROD;
        a.root = 0;
    } else {
        hk = lp_hkind(p, X->dtype == PCF_F64);
        a.root = (kind == PCF_LP_POW || p == 1.0) ? 0 : (p == 2.0 ? 1 : 2);
    }
    e = launch_forward(X->dtype == PCF_F64, hk, a, tile_grid(&plan, false), s);
    if (e != hipSuccess)
        return hip_fail(e, "tile kernel launch");
    return PCF_OK;
}

pcf_status pcf_single(const pcf_set *X, pcf_single_kind kind, double p, double a,
                      double b, void *out, void *stream)
{
    pcf_status st = check_set(X);
    if (st != PCF_OK)
        return st;
    if (kind != PCF_INTEGRAL && kind != PCF_NORM && kind != PCF_NORM_POW &&
        kind != PCF_NORM_INF)
        return fail(PCF_EINVAL, "unknown single-PCF kind");
    if ((kind == PCF_NORM || kind == PCF_NORM_POW) && (!(p >= 1.0) || !isfinite(p)))
        return fail(PCF_EINVAL, "p must be finite and >= 1");
    if (!(a >= 0.0) || !isfinite(a) || !(b > a))
        return fail(PCF_EINVAL, "the bounds must satisfy 0 <= a < b (b may be inf)");
    if (X->n == 0)
        return PCF_OK;
    if (!out)
        return fail(PCF_EINVAL, "out is NULL");
    SingleArgs g;
    g.offsets = X->offsets;
    g.n = X->n;
    g.t = X->t;
    g.v = X->v;
    g.out = out;
    g.a = a;
    g.b = b;
    g.p = p;
    int sk;
    if (kind == PCF_INTEGRAL || kind == PCF_NORM_INF) {
        sk = kind == PCF_INTEGRAL ? 0 : 4;  // segment sum of v, or sup of |v|
        g.root = 0;
    } else {
        sk = p == 1.0 ? 1 : (p == 2.0 ? 2 : 3);
        g.root = (kind == PCF_NORM_POW || p == 1.0) ? 0 : (p == 2.0 ? 1 : 2);
    }
    hipError_t e = launch_single(X->dtype == PCF_F64, sk, g, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "single-PCF kernel launch");
    return PCF_OK;
}

pcf_status pcf_restrict_rows(const pcf_set *X, double a, double b, int64_t *offsets_out,
                             int64_t *offsets_out_host, void *stream)
{
    pcf_status st = check_set(X);
    if (st != PCF_OK)
        return st;
    st = check_range(X, a, b);
    if (st != PCF_OK)
        return st;
    if (!offsets_out || !offsets_out_host)
        return fail(PCF_EINVAL, "offsets_out or offsets_out_host is NULL");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_restrict_count(X->dtype == PCF_F64, X->offsets, X->n, X->t, a, b,
                                         offsets_out, s);
    if (e != hipSuccess)
        return hip_fail(e, "restriction count launch");
    return counts_to_offsets(X->n, offsets_out, offsets_out_host, s, "restricted");
}

pcf_status pcf_restrict(const pcf_set *X, double a, double b, const int64_t *offsets_out,
                        void *t_out, void *v_out, void *stream)
{
    pcf_status st = check_set(X);
    if (st != PCF_OK)
        return st;
    st = check_range(X, a, b);
    if (st != PCF_OK)
        return st;
    if (X->n == 0)
        return PCF_OK;
    if (!offsets_out || !t_out || !v_out)
        return fail(PCF_EINVAL, "an output pointer is NULL");
    hipError_t e = launch_restrict_fill(X->dtype == PCF_F64, X->offsets, X->n, X->t, X->v,
                                        a, b, offsets_out, t_out, v_out,
                                        (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "restriction kernel launch");
    return PCF_OK;
}

pcf_status pcf_warp_rows(const pcf_set *X, pcf_weight_kind weight, double c,
                         int64_t *offsets_out, int64_t *offsets_out_host, void *stream)
{
    pcf_status st = check_set(X);
    if (st == PCF_OK)
        st = check_weight(weight, c);
    if (st != PCF_OK)
        return st;
    if (!offsets_out || !offsets_out_host)
        return fail(PCF_EINVAL, "offsets_out or offsets_out_host is NULL");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_warp_count(X->dtype == PCF_F64, X->offsets, X->n, X->t,
                                     (int)weight, c, offsets_out, s);
    if (e != hipSuccess)
        return hip_fail(e, "warp count launch");
    return counts_to_offsets(X->n, offsets_out, offsets_out_host, s, "warped");
}

pcf_status pcf_warp(const pcf_set *X, pcf_weight_kind weight, double c,
                    const int64_t *offsets_out, void *t_out, void *v_out, void *stream)
{
    pcf_status st = check_set(X);
    if (st == PCF_OK)
        st = check_weight(weight, c);
    if (st != PCF_OK)
        return st;
    if (X->n == 0)
        return PCF_OK;
    if (!offsets_out || !t_out || !v_out)
        return fail(PCF_EINVAL, "an output pointer is NULL");
    hipError_t e = launch_warp_fill(X->dtype == PCF_F64, X->offsets, X->n, X->t, X->v,
                                    (int)weight, c, offsets_out, t_out, v_out,
                                    (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "warp kernel launch");
    return PCF_OK;
}

pcf_status pcf_restrict_backward(const pcf_set *X, double a, double b,
                                 const int64_t *offsets_y, const void *grad_t_y,
                                 const void *grad_v_y, void *grad_t_x, void *grad_v_x,
                                 void *stream)
{
    pcf_status st = check_set(X);
    if (st == PCF_OK)
        st = check_range(X, a, b);
    if (st != PCF_OK)
        return st;
    if (X->n == 0)
        return PCF_OK;
    if (!offsets_y || !grad_t_y || !grad_v_y || !grad_t_x || !grad_v_x)
        return fail(PCF_EINVAL, "a gradient or offsets pointer is NULL");
    hipError_t e = launch_restrict_backward(
        X->dtype == PCF_F64, X->offsets, X->n, X->t, a, b, offsets_y,
        (const double *)grad_t_y, (const double *)grad_v_y, (double *)grad_t_x,
        (double *)grad_v_x, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "restriction gradient launch");
    return PCF_OK;
}

pcf_status pcf_warp_backward(const pcf_set *X, pcf_weight_kind weight, double c,
                             const int64_t *offsets_y, const void *grad_t_y,
                             const void *grad_v_y, void *grad_t_x, void *grad_v_x,
                             void *stream)
{
    pcf_status st = check_set(X);
    if (st == PCF_OK)
        st = check_weight(weight, c);
    if (st != PCF_OK)
        return st;
    if (X->n == 0)
        return PCF_OK;
    if (!offsets_y || !grad_t_y || !grad_v_y || !grad_t_x || !grad_v_x)
        return fail(PCF_EINVAL, "a gradient or offsets pointer is NULL");
    hipError_t e = launch_warp_backward(
        X->dtype == PCF_F64, X->offsets, X->n, X->t, (int)weight, c, offsets_y,
        (const double *)grad_t_y, (const double *)grad_v_y, (double *)grad_t_x,
        (double *)grad_v_x, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "warp gradient launch");
    return PCF_OK;
}

pcf_status pcf_reduce_workspace_bytes(const pcf_set *X, int32_t B,
                                      const int64_t *group_offsets_host, pcf_reduce_op op,
                                      size_t *bytes)
{
    if (!bytes)
        return fail(PCF_EINVAL, "bytes is NULL");
    if (op < PCF_REDUCE_SUM || op > PCF_REDUCE_STD)
        return fail(PCF_EINVAL, "unknown reduction op");
    RedPlan rp;
    pcf_status st = red_plan(X, B, group_offsets_host, (int)op, nullptr, rp);
    if (st != PCF_OK)
        return st;
    *bytes = rp.bytes;
    return PCF_OK;
}

namespace {

// The sum tree's roots (or the set itself when no group has two PCFs).
void red_roots(const pcf_set *X, const RedPlan &rp, unsigned char *w, const void *&rt,
               const void *&rv)
{
    if (rp.L == 0) {
        rt = X->t;
        rv = X->v;
    } else {
        const int k = (rp.L - 1) % 2;
        rt = w + rp.off_buf[2 * k];
        rv = w + rp.off_buf[2 * k + 1];
    }
}

}  // namespace

static pcf_status reduce_rows_impl(const pcf_set *X, int32_t B,
                                   const int64_t *group_offsets_host, int op, void *ws,
                                   size_t ws_bytes, int64_t *offsets_out,
                                   int64_t *offsets_out_host, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    RedPlan rp;
    pcf_status st = red_plan(X, B, group_offsets_host, (int)op, s, rp);
    if (st != PCF_OK)
        return st;
    if (!offsets_out || !offsets_out_host)
        return fail(PCF_EINVAL, "offsets_out or offsets_out_host is NULL");
    if (B == 0)
        return counts_to_offsets(0, offsets_out, offsets_out_host, s, "reduced");
    if (!ws || ws_bytes < rp.bytes)
        return fail(PCF_ENOMEM, "workspace too small: need " + std::to_string(rp.bytes) +
                                    " bytes, got " + std::to_string(ws_bytes));
    unsigned char *w = (unsigned char *)ws;
    int64_t *meta = (int64_t *)w;
    hipError_t e = hipMemcpyAsync(meta, rp.meta.data(), rp.meta.size() * sizeof(int64_t),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);  // rp.meta is a local
    const bool f64 = X->dtype == PCF_F64;
    int32_t *row_pcf = (int32_t *)(w + rp.off_map);
    if (e == hipSuccess && rp.L > 0)
        e = launch_red_rowmap(X->offsets, rp.n, row_pcf, s);
    for (int l = 0; l < rp.L && e == hipSuccess; ++l) {
        RedLevelArgs a;
        a.offsets = X->offsets;
        a.groups = meta;
        a.row_pcf = row_pcf;
        a.n = rp.n;
        a.B = B;
        a.level = l;
        const int ki = (l + 1) % 2, ko = l % 2;  // level l writes buffer pair l % 2
        a.tin = l == 0 ? X->t : (const void *)(w + rp.off_buf[2 * ki]);
        a.vin = l == 0 ? X->v : (const void *)(w + rp.off_buf[2 * ki + 1]);
        a.tout = w + rp.off_buf[2 * ko];
        a.vout = w + rp.off_buf[2 * ko + 1];
        e = launch_red_level(f64, (int)op, a, rp.P, s);
    }
    const void *rt, *rv;
    red_roots(X, rp, w, rt, rv);
    if (e == hipSuccess && op == RO_STD) {
        RedStdArgs a;
        a.offsets = X->offsets;
        a.groups = meta;
        a.B = B;
        a.rows = rp.P;
        a.t = X->t;
        a.v = X->v;
        a.rt = rt;
        a.rv = rv;
        a.q = w + rp.off_q;
        a.nchunks = rp.C;
        a.chunk_row = meta + B + 1;
        a.chunk_grp = meta + B + 1 + rp.C;
        a.chunk_first = (int64_t *)(w + rp.off_kb);
        // groups of at most 64 PCFs by red_std_small, larger ones (if any)
        // by red_std_terms
        bool large = false;
        for (int32_t b = 0; b < B && !large; ++b)
            large = group_offsets_host[b + 1] - group_offsets_host[b] > 64;
        e = launch_red_std_small(f64, a, s);
        if (e == hipSuccess && large)
            e = launch_red_std(f64, a, s);
        rv = w + rp.off_q;
    }
    int64_t *ccnt = (int64_t *)(w + rp.off_ccnt), *coff = (int64_t *)(w + rp.off_coff);
    if (e == hipSuccess) {
        RedEmitArgs a;
        a.offsets = X->offsets;
        a.groups = meta;
        a.op = (int)op;
        a.rt = rt;
        a.rv = rv;
        a.nchunks = rp.C;
        a.chunk_row = meta + B + 1;
        a.chunk_grp = meta + B + 1 + rp.C;
        a.fill = 0;
        a.chunk_cnt = ccnt;
        a.chunk_off = nullptr;
        a.out_end = nullptr;
        a.t_out = a.v_out = nullptr;
        e = launch_red_emit(f64, a, s);
    }
    std::vector<int64_t> cc((size_t)rp.C);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cc.data(), ccnt, sizeof(int64_t) * (size_t)rp.C,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "reduction launch");
    // chunk counts -> chunk output offsets (chunks are in group order) and
    // per-group offsets
    const int64_t *cgrp = rp.meta.data() + B + 1 + rp.C;
    std::vector<int64_t> gc((size_t)B, 0);
    int64_t acc = 0;
    for (int64_t c = 0; c < rp.C; ++c) {
        const int64_t k = cc[(size_t)c];
        cc[(size_t)c] = acc;
        acc += k;
        gc[(size_t)cgrp[c]] += k;
    }
    offsets_out_host[0] = 0;
    for (int32_t b = 0; b < B; ++b)
        offsets_out_host[b + 1] = offsets_out_host[b] + gc[(size_t)b];
    e = hipMemcpyAsync(coff, cc.data(), sizeof(int64_t) * (size_t)rp.C, hipMemcpyHostToDevice,
                       s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(offsets_out, offsets_out_host, sizeof(int64_t) * (size_t)(B + 1),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);  // cc and offsets_out_host may be locals
    return e == hipSuccess ? PCF_OK : hip_fail(e, "writing the reduced offsets");
}

static pcf_status reduce_fill_impl(const pcf_set *X, int32_t B,
                                   const int64_t *group_offsets_host, int op, const void *ws,
                                   size_t ws_bytes, const int64_t *offsets_out, void *t_out,
                                   void *v_out, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    RedPlan rp;
    pcf_status st = red_plan(X, B, group_offsets_host, (int)op, s, rp);
    if (st != PCF_OK)
        return st;
    if (B == 0)
        return PCF_OK;
    if (!ws || ws_bytes < rp.bytes)
        return fail(PCF_ENOMEM, "workspace too small");
    if (!offsets_out || !t_out || !v_out)
        return fail(PCF_EINVAL, "an output pointer is NULL");
    unsigned char *w = (unsigned char *)ws;
    const int64_t *meta = (const int64_t *)w;
    const void *rt, *rv;
    red_roots(X, rp, w, rt, rv);
    RedEmitArgs a;
    a.offsets = X->offsets;
    a.groups = meta;
    a.op = (int)op;
    a.rt = rt;
    a.rv = op == RO_STD ? (const void *)(w + rp.off_q) : rv;
    a.nchunks = rp.C;
    a.chunk_row = meta + B + 1;
    a.chunk_grp = meta + B + 1 + rp.C;
    a.fill = 1;
    a.chunk_cnt = nullptr;
    a.chunk_off = (const int64_t *)(w + rp.off_coff);
    a.out_end = offsets_out + B;
    a.t_out = t_out;
    a.v_out = v_out;
    hipError_t e = launch_red_emit(X->dtype == PCF_F64, a, s);
    if (e != hipSuccess)
        return hip_fail(e, "reduction launch");
    return PCF_OK;
}

pcf_status pcf_reduce_rows(const pcf_set *X, int32_t B, const int64_t *group_offsets_host,
                           pcf_reduce_op op, void *ws, size_t ws_bytes, int64_t *offsets_out,
                           int64_t *offsets_out_host, void *stream)
{
    if (op < PCF_REDUCE_SUM || op > PCF_REDUCE_STD)
        return fail(PCF_EINVAL, "unknown reduction op");
    return reduce_rows_impl(X, B, group_offsets_host, (int)op, ws, ws_bytes, offsets_out,
                            offsets_out_host, stream);
}

pcf_status pcf_reduce(const pcf_set *X, int32_t B, const int64_t *group_offsets_host,
                      pcf_reduce_op op, const void *ws, size_t ws_bytes,
                      const int64_t *offsets_out, void *t_out, void *v_out, void *stream)
{
    if (op < PCF_REDUCE_SUM || op > PCF_REDUCE_STD)
        return fail(PCF_EINVAL, "unknown reduction op");
    return reduce_fill_impl(X, B, group_offsets_host, (int)op, ws, ws_bytes, offsets_out,
                            t_out, v_out, stream);
}

}  // extern "C"

namespace {

// A combination of X and Y as a reduction of Z = (X_0, Y_0, X_1, Y_1, ...)
// in groups of two; Z's offsets and rows sit at the head of the workspace.
struct CombPlan {
    int64_t n = 0;
    std::vector<int64_t> zoff, groups;
    size_t off_zt = 0, off_zv = 0, off_red = 0, bytes = 0;
    int ro = RO_SUM;
    pcf_set Z{};
    RedPlan rp;
};

int combine_ro(int op)
{
    switch (op) {
    case PCF_COMBINE_SUM: return RO_SUM;
    case PCF_COMBINE_SUB: return RO_SUB;
    case PCF_COMBINE_MUL: return RO_MUL;
    case PCF_COMBINE_MAX: return RO_MAX;
    case PCF_COMBINE_MIN: return RO_MIN;
    case PCF_COMBINE_SQDIFF: return RO_SQDIFF;
    default: return -1;
    }
}

pcf_status comb_plan(const pcf_set *X, const pcf_set *Y, int op, unsigned char *ws,
                     hipStream_t s, CombPlan &cp)
{
    pcf_status st = check_pair(X, Y);
    if (st != PCF_OK)
        return st;
    if (X->n != Y->n)
        return fail(PCF_EINVAL, "X and Y must hold the same number of PCFs");
    cp.ro = combine_ro(op);
    if (cp.ro < 0)
        return fail(PCF_EINVAL, "unknown combination op");
    const int64_t n = X->n;
    if (n >= ((int64_t)1 << 30))
        return fail(PCF_EUNSUPPORTED, "combinations take fewer than 2^30 PCFs");
    std::vector<int64_t> xb, yb;
    const int64_t *xo = nullptr, *yo = nullptr;
    if (n > 0) {
        st = host_offsets(X, xb, xo, s);
        if (st == PCF_OK)
            st = host_offsets(Y, yb, yo, s);
        if (st != PCF_OK)
            return st;
    }
    cp.n = n;
    cp.zoff.assign((size_t)(2 * n + 1), 0);
    cp.groups.assign((size_t)(n + 1), 0);
    for (int64_t i = 0; i < n; ++i) {
        cp.zoff[(size_t)(2 * i + 1)] = cp.zoff[(size_t)(2 * i)] + (xo[i + 1] - xo[i]);
        cp.zoff[(size_t)(2 * i + 2)] = cp.zoff[(size_t)(2 * i + 1)] + (yo[i + 1] - yo[i]);
        cp.groups[(size_t)(i + 1)] = 2 * (i + 1);
    }
    const int64_t P = cp.zoff.back();
    const size_t esz = X->dtype == PCF_F64 ? 8 : 4;
    size_t off = align256(cp.zoff.size() * sizeof(int64_t));
    cp.off_zt = off;
    off += align256((size_t)(P > 0 ? P : 1) * esz);
    cp.off_zv = off;
    off += align256((size_t)(P > 0 ? P : 1) * esz);
    cp.off_red = off;
    cp.Z.n = 2 * n;
    // without a workspace (a size query) X's pointers stand in; the plan
    // reads only Z's host offsets
    cp.Z.offsets = ws ? (const int64_t *)ws : X->offsets;
    cp.Z.t = ws ? (const void *)(ws + cp.off_zt) : X->t;
    cp.Z.v = ws ? (const void *)(ws + cp.off_zv) : X->v;
    cp.Z.dtype = X->dtype;
    cp.Z.offsets_host = cp.zoff.data();
    if (n > 0) {
        st = red_plan(&cp.Z, (int32_t)n, cp.groups.data(), cp.ro, s, cp.rp);
        if (st != PCF_OK)
            return st;
    }
    cp.bytes = off + cp.rp.bytes;
    return PCF_OK;
}

}  // namespace

extern "C" {

pcf_status pcf_combine_workspace_bytes(const pcf_set *X, const pcf_set *Y, pcf_combine_op op,
                                       size_t *bytes)
{
    if (!bytes)
        return fail(PCF_EINVAL, "bytes is NULL");
    CombPlan cp;
    pcf_status st = comb_plan(X, Y, (int)op, nullptr, nullptr, cp);
    if (st != PCF_OK)
        return st;
    *bytes = cp.bytes;
    return PCF_OK;
}

pcf_status pcf_combine_rows(const pcf_set *X, const pcf_set *Y, pcf_combine_op op, void *ws,
                            size_t ws_bytes, int64_t *offsets_out, int64_t *offsets_out_host,
                            void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    unsigned char *w = (unsigned char *)ws;
    CombPlan cp;
    pcf_status st = comb_plan(X, Y, (int)op, w, s, cp);
    if (st != PCF_OK)
        return st;
    if (!offsets_out || !offsets_out_host)
        return fail(PCF_EINVAL, "offsets_out or offsets_out_host is NULL");
    if (cp.n == 0)
        return counts_to_offsets(0, offsets_out, offsets_out_host, s, "combined");
    if (!w || ws_bytes < cp.bytes)
        return fail(PCF_ENOMEM, "workspace too small: need " + std::to_string(cp.bytes) +
                                    " bytes, got " + std::to_string(ws_bytes));
    hipError_t e = hipMemcpyAsync(w, cp.zoff.data(), cp.zoff.size() * sizeof(int64_t),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);  // cp.zoff is a local
    if (e == hipSuccess)
        e = launch_red_interleave(X->dtype == PCF_F64, cp.n, X->offsets, X->t, X->v,
                                  Y->offsets, Y->t, Y->v, (const int64_t *)w, w + cp.off_zt,
                                  w + cp.off_zv, s);
    if (e != hipSuccess)
        return hip_fail(e, "combination launch");
    return reduce_rows_impl(&cp.Z, (int32_t)cp.n, cp.groups.data(), cp.ro, w + cp.off_red,
                            ws_bytes - cp.off_red, offsets_out, offsets_out_host, stream);
}

pcf_status pcf_combine(const pcf_set *X, const pcf_set *Y, pcf_combine_op op, const void *ws,
                       size_t ws_bytes, const int64_t *offsets_out, void *t_out, void *v_out,
                       void *stream)
{
    unsigned char *w = (unsigned char *)ws;
    CombPlan cp;
    pcf_status st = comb_plan(X, Y, (int)op, w, (hipStream_t)stream, cp);
    if (st != PCF_OK)
        return st;
    if (cp.n == 0)
        return PCF_OK;
    if (!w || ws_bytes < cp.bytes)
        return fail(PCF_ENOMEM, "workspace too small");
    return reduce_fill_impl(&cp.Z, (int32_t)cp.n, cp.groups.data(), cp.ro, w + cp.off_red,
                            ws_bytes - cp.off_red, offsets_out, t_out, v_out, stream);
}

}  // extern "C"
