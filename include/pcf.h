/*
 * pcf.h -- C ABI of the MI355X (gfx950) library for pairwise integrated
 * combinations of piecewise constant functions (PCFs).
 *
 * What is computed (paper: Section 1 defines d_p and <.,.>; Section 2.2
 * "Functionals" defines combination integrals F(f,g) = r(int h(f,g) dt);
 * Section 3, Eq. "simpleint", sums h over the cells of a common
 * discretization; Section 3.1 defines the pairwise matrix F(C) with
 * F_ij = F(f_i, f_j); Algorithms "IterateRectangles" and
 * "CombineIntegrate" walk both breakpoint lists once):
 *
 *   PCF_LP      F = (int |f-g|^p)^(1/p)       L_p distance, p >= 1
 *   PCF_LP_POW  F =  int |f-g|^p              d_p^p (no root)
 *   PCF_GRAM    F =  int f g                  L2 inner product
 *
 * Data layout (ragged CSR, structure of arrays). A set of n PCFs is
 *   offsets[n+1]  int64, offsets[0] = 0, PCF i owns rows
 *                 offsets[i] .. offsets[i+1]-1;
 *   t[P], v[P]    breakpoint times and values, both FP32 or both FP64,
 *                 P = offsets[n].
 * Every PCF has between 1 and 2^30 - 1 rows; the planner rejects other row
 * counts with PCF_EINVAL (an empty PCF, or one so long that a pair's merge
 * could exceed 2^31 steps).
 * PCF i is f(x) = v[k] for t[k] <= x < t[k+1] (rows k of PCF i) and
 * v[last] after the last time (paper, Section 2; its n x 2 matrix [t; f]).
 * Contract (checked only under PCF_VALIDATE): every PCF has >= 1 row, its
 * first time is 0, its times strictly increase, all values are finite and
 * its last value is 0 (eventually zero, so integrals over [0, inf) are
 * finite). Unchecked violations give unspecified results, never a fault.
 *
 * Conventions.
 *  - Every pointer inside pcf_set and every data/output/workspace pointer is
 *    a DEVICE pointer, except pcf_set.offsets_host (optional HOST copy of
 *    offsets; when NULL the library copies offsets to the host itself and
 *    synchronises the stream). The caller owns every buffer; the library
 *    keeps no pointer after a call returns and allocates no device memory.
 *  - Calls are asynchronous on `stream` (a hipStream_t, NULL = default
 *    stream) except where a host copy or a validation forces a
 *    synchronisation, as documented per call.
 *  - Output dtype equals input dtype. Output is row-major with leading
 *    dimension `ldo` (elements). A window (rows [row0,row1) x columns
 *    [col0,col1)) writes entry (i,j) at out[(i-row0)*ldo + (j-col0)]; NULL
 *    means the full n x n matrix. Entries for which both (i,j) and (j,i) lie
 *    in the window are computed once and written to both places, bit for bit
 *    equal. Distance diagonals are exactly 0; the Gram diagonal is int f_i^2.
 *  - The workspace `ws` (device, 256-byte aligned, at least the size returned
 *    by pcf_workspace_bytes) holds the packed breakpoint records, the tile
 *    plan and the tile counter. With PCF_REUSE_PLAN the plan already in `ws`
 *    (from an earlier call on a set with identical offsets, window and kind)
 *    is reused and the call performs no host<->device copy and no
 *    synchronisation: it only launches kernels on `stream`, so it may be
 *    captured into a HIP graph.
 *  - No exception crosses the ABI. A non-OK status leaves a message for
 *    pcf_last_error() (thread-local).
 *  - Calls that overlap on one device and share a workspace race; give each
 *    concurrent call its own workspace.
 */
#ifndef PCF_H
#define PCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PCF_OK = 0,
    PCF_EINVAL = 1,       /* bad argument (null pointer, size, p, window) */
    PCF_EDATA = 2,        /* contract violation found by PCF_VALIDATE     */
    PCF_EDEVICE = 3,      /* HIP runtime error                            */
    PCF_ENOMEM = 4,       /* workspace too small                          */
    PCF_EUNSUPPORTED = 5  /* valid request the library does not serve    */
} pcf_status;

typedef enum { PCF_F32 = 0, PCF_F64 = 1 } pcf_dtype;

typedef enum {
    PCF_LP = 0,     /* (int |f-g|^p)^(1/p)  */
    PCF_LP_POW = 1, /*  int |f-g|^p         */
    PCF_GRAM = 2    /*  int f g             */
} pcf_kind;

typedef struct {
    int64_t n;                    /* number of PCFs                          */
    const int64_t *offsets;       /* device, n+1                             */
    const void *t;                /* device, offsets[n] times                */
    const void *v;                /* device, offsets[n] values               */
    pcf_dtype dtype;              /* of t, v and of the output               */
    const int64_t *offsets_host;  /* optional host copy of offsets, or NULL  */
} pcf_set;

typedef struct {
    int64_t row0, row1, col0, col1; /* half-open PCF index ranges */
} pcf_window;

enum {
    PCF_UPPER_ONLY = 1u,    /* write only (i,j) with i <= j of symmetric parts */
    PCF_VALIDATE = 2u,      /* check the data contract first (synchronises)   */
    PCF_DETERMINISTIC = 4u, /* bit-identical results run to run for a given
                                plan: always true of the matrix calls
                                (fixed-order partial sums); for
                                pcf_pairwise_backward, integer gradient sums
                                (see there)                                 */
    PCF_REUSE_PLAN = 8u,    /* reuse the plan already in ws (see above)       */
    PCF_RECORDS_PACKED = 16u /* with PCF_REUSE_PLAN: ws also still holds the
                                packed records of these very t and v (e.g. an
                                L1 then a Gram matrix of one set): skip the
                                packing pass                                  */
};

/* Tile shape (chosen by an autotuner; 0 = default). Bits 8..13 of `flags`:
 * most PCFs per block (1..32, default 32); bits 16..19: a block holds at most
 * 1/d of a tile's LDS record capacity (d = 2..8, default 2). Results are the
 * same for every shape up to rounding order. */
#define PCF_TILE_SHAPE(max_block, budget_div) \
    ((((uint32_t)(max_block) & 63u) << 8) | (((uint32_t)(budget_div) & 15u) << 16))

/* Workspace size in bytes for pcf_pairwise_lp / pcf_gram (backward = 0) or
 * pcf_pairwise_backward (backward = 1) on X with window w (NULL = full),
 * enough for every tile shape.
 * Reads X->offsets (host copy or a synchronous device-to-host copy).
 * Returns PCF_EINVAL on bad arguments. */
pcf_status pcf_workspace_bytes(const pcf_set *X, pcf_kind kind,
                               const pcf_window *w, int backward,
                               size_t *bytes);

/* L_p distance matrix of X (PCF_LP, p >= 1) or its p-th power
 * (PCF_LP_POW): out[i][j] = F(f_i, f_j) (Section 3.1 with h = |a-b|^p,
 * Section 2.2). p = 1 and p = 2 use exact products, other integer p
 * squaring; in FP64 p = k + 1/2 adds one square root and any other p is
 * 2^(p log2 |a-b|) by a series (relative error within a few units of the
 * last place times |p log2 |a-b||), in FP32 every non-integer p uses the
 * hardware base-2 log and exp.
 * Errors: PCF_EINVAL (null pointers, n < 0, p < 1 or not finite, bad
 * window, ldo too small, kind not an L_p kind), PCF_ENOMEM (ws_bytes too
 * small), PCF_EDATA (PCF_VALIDATE found a violation; the index of the first
 * bad PCF is in pcf_last_error()), PCF_EDEVICE. */
pcf_status pcf_pairwise_lp(const pcf_set *X, pcf_kind kind, double p,
                           void *out, int64_t ldo, const pcf_window *w,
                           void *ws, size_t ws_bytes, uint32_t flags,
                           void *stream);

/* L2 Gram matrix: out[i][j] = int f_i f_j (Section 2.2, h = ab, r = id).
 * Same arguments and errors as pcf_pairwise_lp. */
pcf_status pcf_gram(const pcf_set *X, void *out, int64_t ldo,
                    const pcf_window *w, void *ws, size_t ws_bytes,
                    uint32_t flags, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * pcf_pairwise_lp (kind PCF_LP or PCF_LP_POW) and pcf_gram (kind PCF_GRAM)
 * with the workspace taken from a device array the library holds, of
 * PCF_NOALLOC_SCRATCH_BYTES bytes on every GPU it runs on (held from module
 * load until the process ends), instead of a caller buffer. Same arguments,
 * results and errors as pcf_pairwise_lp, without ws and ws_bytes; calls no
 * allocating routine. PCF_ENOMEM (before any device work when
 * X->offsets_host is given) when the call's plan and packed records exceed
 * the array; PCF_EINVAL for PCF_REUSE_PLAN or PCF_RECORDS_PACKED, since every
 * call on a device shares that device's array and overwrites what it held.
 * Calls that overlap on one device (other streams or host threads) race;
 * calls in one stream are ordered. */
#define PCF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
pcf_status pcf_pairwise_lp_noalloc(const pcf_set *X, pcf_kind kind, double p,
                                   void *out, int64_t ldo, const pcf_window *w,
                                   uint32_t flags, void *stream);

/* Adjoint of a full-matrix call (not in the paper; the paper's Section 3
 * aside only notes that derivatives are analytic). Given grad_out = dL/dF
 * (n x n, leading dimension ldg) and, for PCF_LP with p != 1, the forward
 * result fwd_out (n x n, leading dimension ldf; may be NULL otherwise),
 * writes dL/dt into grad_t and dL/dv into grad_v (device, P entries each,
 * same CSR layout and dtype as t and v; overwritten). Uses
 * w_ij = grad_out[i][j] + grad_out[j][i] for i < j and grad_out[i][i] on the
 * diagonal. The first time and the last value of every PCF are fixed: their
 * entries are 0. At an exact tie of two PCFs' breakpoint times the mean of
 * the one-sided time derivatives is used. Each pair's merge is recomputed;
 * nothing is stored between forward and backward. grad_out and fwd_out are
 * FP64 for either dtype, and finite (the fixed-point sums below are scaled
 * from their magnitudes; a NaN or infinite weight gives undefined
 * gradients rather than NaN ones); an FP32 set merges and forms its gradient
 * terms in FP32. A tile sums its gradient terms in 64-bit fixed point at power-of-two
 * scales bounded from its own weights, values and piece lengths
 * (order-independent), and adds the sums to grad_t, grad_v with atomics of
 * the set's dtype, whose order, and so the last bits, may vary between runs.
 * With PCF_DETERMINISTIC the sums in HBM are 64-bit fixed point too (for
 * FP32 sets in the workspace, which pcf_workspace_bytes with backward = 1
 * sizes for it), at
 * scales bounded from the whole set (largest |w_ij|, |v| and piece length,
 * found by two extra passes over grad_out, fwd_out and the records), until a
 * last pass converts them into grad_t and grad_v,
 * and the result is bit-identical run to run for a given plan and tile
 * shape. Each term is then rounded to a unit of about 2^-61 (n + 1) times
 * the set's largest possible term, so gradients far below that lose
 * relative precision. PCF_EUNSUPPORTED for more than 2,097,120 PCFs with
 * PCF_DETERMINISTIC. */
pcf_status pcf_pairwise_backward(const pcf_set *X, pcf_kind kind, double p,
                                 const void *grad_out, int64_t ldg,
                                 const void *fwd_out, int64_t ldf,
                                 void *grad_t, void *grad_v, void *ws,
                                 size_t ws_bytes, uint32_t flags,
                                 void *stream);

/* Cross-set matrix of two collections X (rows) and Y (columns): entry
 * (i, j) is F(X_i, Y_j) for the combination integral F of Section 2.2 (the
 * pairwise matrix of Section 3.1 taken over two collections instead of one,
 * e.g. test against training PCFs), written at out[i*ldo + j] (ldo >= Y->n).
 * kind and p as in pcf_pairwise_lp, or PCF_GRAM (p ignored). X and Y share
 * their dtype. The library copies both offset arrays to the host unless
 * offsets_host is given, plans the X x Y rectangle over one CSR of X then Y,
 * and packs both sets' records into one array of the workspace (size from
 * pcf_cross_workspace_bytes). Flags: PCF_VALIDATE and the tile shape;
 * PCF_UPPER_ONLY, PCF_REUSE_PLAN and PCF_RECORDS_PACKED give PCF_EINVAL.
 * Errors as pcf_pairwise_lp (PCF_EDATA names the set and PCF). */
pcf_status pcf_cross(const pcf_set *X, const pcf_set *Y, pcf_kind kind, double p,
                     void *out, int64_t ldo, void *ws, size_t ws_bytes,
                     uint32_t flags, void *stream);

/* Workspace size for pcf_cross on X and Y, enough for every tile shape. */
pcf_status pcf_cross_workspace_bytes(const pcf_set *X, const pcf_set *Y,
                                     size_t *bytes);

/* Functionals of one PCF at a time (paper, Section 3.2 "PCF integrals"):
 *   F(f) = r( int_a^b h(f(t)) dt ),   0 <= a < b <= inf (b may be INFINITY),
 * by segment iteration (Algorithm IterateSegments):
 *   PCF_INTEGRAL  h(v) = v                         (p ignored)
 *   PCF_NORM      h(v) = |v|^p, r(x) = x^(1/p)     (the L_p norm, p >= 1)
 *   PCF_NORM_POW  h(v) = |v|^p, r(x) = x
 *   PCF_NORM_INF  sup over [a, b) of |f| (the largest |v| of the segments
 *                 the iteration lists; p ignored)
 * out[i] (n entries of X's dtype, device) = F(f_i). With b = inf a nonzero
 * last value gives an infinity of the sign of h. Asynchronous on `stream`;
 * no workspace, no host copy. PCF_EINVAL on bad arguments (bounds, p,
 * kind, NULL pointers). */
typedef enum {
    PCF_INTEGRAL = 0,
    PCF_NORM = 1,
    PCF_NORM_POW = 2,
    PCF_NORM_INF = 3
} pcf_single_kind;

pcf_status pcf_single(const pcf_set *X, pcf_single_kind kind, double p, double a,
                      double b, void *out, void *stream);

/* Restriction to an integration range (Section 2.2: combination integrals
 * over [a, b), 0 <= a < b <= inf). f 1_[a,b) is a PCF again, and h(0,0) = 0
 * for every kind, so any entry point run on the restricted set computes its
 * integrals over [a, b) (e.g. pcf_pairwise_lp gives (int_a^b |f-g|^p)^(1/p)).
 * Rows of the restriction of f: (0, 0) and (a, f(a)) when a > 0, else
 * (0, f(0)); the rows of f with a < t_k < b; (b, 0) when b is finite. a and
 * b are rounded to the set's dtype and must stay ordered (PCF_EINVAL).
 * Two calls: pcf_restrict_rows writes the restricted set's offsets to
 * offsets_out (device, n+1) and to offsets_out_host (host, n+1), and
 * synchronises; the caller then allocates t_out and v_out with
 * offsets_out_host[n] entries of X's dtype and calls pcf_restrict
 * (asynchronous), which fills them. */
pcf_status pcf_restrict_rows(const pcf_set *X, double a, double b, int64_t *offsets_out,
                             int64_t *offsets_out_host, void *stream);
pcf_status pcf_restrict(const pcf_set *X, double a, double b, const int64_t *offsets_out,
                        void *t_out, void *v_out, void *stream);

/* Time-dependent combinations (Section 3: h(a, b, t) with an antiderivative
 * H in t; Section 2.2: weighted L_p distance and weighted inner product).
 * For h = h0(a, b) w(t) every cell [l, r) of the merge adds
 * h0 (W(r) - W(l)), W(t) = int_0^t w. pcf_warp carries each breakpoint t_k
 * to tau_k = W(t_k), so every entry point run on the warped set computes the
 * weighted integrals (pcf_pairwise_lp gives (int |f-g|^p w)^(1/p)); with a
 * range, restrict first, then warp. Weights (c is the parameter):
 *   PCF_WEIGHT_EXP  w(t) = exp(-c t), c > 0    W(t) = (1 - exp(-c t)) / c
 *   PCF_WEIGHT_POW  w(t) = t^c, c > -1         W(t) = t^(c+1) / (c+1)
 * W is computed in FP64 and rounded to the set's dtype; rows whose rounded
 * tau ties with the next row's are dropped (the later row's value holds on
 * the next piece), so the warped set is again strictly increasing. A tau
 * that overflows gives PCF_EINVAL naming the PCF. Two calls, as for the
 * restriction: pcf_warp_rows writes the warped offsets to offsets_out
 * (device, n+1) and offsets_out_host (host, n+1) and synchronises;
 * pcf_warp (asynchronous) fills t_out and v_out, offsets_out_host[n]
 * entries of X's dtype each, allocated by the caller. */
typedef enum {
    PCF_WEIGHT_EXP = 1,
    PCF_WEIGHT_POW = 2
} pcf_weight_kind;

pcf_status pcf_warp_rows(const pcf_set *X, pcf_weight_kind weight, double c,
                         int64_t *offsets_out, int64_t *offsets_out_host, void *stream);
pcf_status pcf_warp(const pcf_set *X, pcf_weight_kind weight, double c,
                    const int64_t *offsets_out, void *t_out, void *v_out, void *stream);

/* Time-dependent combinations given by a sum of separable terms (Section 3:
 * a time-dependent h whose antiderivative H in t is known adds, per
 * rectangle [l, r) with values (a, b), H(a, b, r) - H(a, b, l)). Here
 *   h(a, b, t) = sum_m coef_m h0_m(a, b) w_m(t),  H = sum_m coef_m h0_m W_m,
 * with h0_m = |a - b|^p (PCF_LP_POW) or a b (PCF_GRAM) and w_m = 1 (weight
 * 0), e^{-ct} or t^c (pcf_weight_kind, as pcf_warp): not separable in
 * general. The result is F_ij = r(sum_m coef_m I_m(f_i, f_j)), r(x) = x^(1/q)
 * (q >= 1; q = 0: no root), each I_m on the set warped by w_m. Output and
 * window as pcf_pairwise_lp; PCF_UPPER_ONLY honoured; PCF_REUSE_PLAN and
 * PCF_RECORDS_PACKED refused (PCF_EINVAL: every term plans and packs its own
 * set). A root of a negative sum is NaN. Workspace: pcf_terms_workspace_bytes
 * (the forward's, plus one warped copy of the set). Synchronises the stream
 * once per weighted term (to read the warped row counts). PCF_EINVAL for an
 * empty term list, a bad kind, p, weight or root, or a non-finite
 * coefficient. */
typedef struct {
    pcf_kind kind;           /* PCF_LP_POW or PCF_GRAM */
    double p;                /* the exponent of PCF_LP_POW */
    int weight;              /* 0 (w = 1), PCF_WEIGHT_EXP or PCF_WEIGHT_POW */
    double c;                /* the weight's parameter */
    double coef;             /* the term's coefficient */
} pcf_term;
pcf_status pcf_terms_workspace_bytes(const pcf_set *X, const pcf_window *w, uint32_t flags,
                                     size_t *bytes);
pcf_status pcf_pairwise_terms(const pcf_set *X, int32_t nterms, const pcf_term *terms,
                              double q, void *out, int64_t ldo, const pcf_window *w,
                              void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/* Gradients through a range restriction and a time warp (Section 3, the
 * remark after Algorithm "CombineIntegrate" that the integrals' parameter
 * derivatives are analytic; Section 2.2 ranges and weights). For a loss of a
 * matrix computed on Y = pcf_restrict(X, a, b) or Y = pcf_warp(X, weight, c),
 * these map dL/dt and dL/dv of Y's rows (FP64 device arrays of
 * offsets_y[n] entries each, e.g. from pcf_pairwise_backward on Y; offsets_y
 * the device offsets that pcf_restrict_rows / pcf_warp_rows wrote) to those
 * of X's rows (FP64 device arrays of X's row count, overwritten). With a
 * range and a weight, apply the warp's map, then the restriction's.
 *
 * Restriction: a row of X kept in Y passes its two gradients on; the row
 * holding a receives the value gradient of Y's row (a, v); the times 0, a
 * and b, the added values, every row outside [a, b) and the last value of
 * each PCF (a fixed parameter, as in pcf_pairwise_backward) get 0.
 * Warp (tau = W(t)): dL/dt_k = dL/dtau_k * w(t_k) (W' = w), dL/dv_k as given;
 * t_0 and a row dropped because its rounded tau ties the next get 0.
 * a, b, weight and c must be those of the forward call (PCF_EINVAL as there);
 * PCF_EINVAL for NULL pointers. Asynchronous on `stream`. */
pcf_status pcf_restrict_backward(const pcf_set *X, double a, double b,
                                 const int64_t *offsets_y, const void *grad_t_y,
                                 const void *grad_v_y, void *grad_t_x, void *grad_v_x,
                                 void *stream);
pcf_status pcf_warp_backward(const pcf_set *X, pcf_weight_kind weight, double c,
                             const int64_t *offsets_y, const void *grad_t_y,
                             const void *grad_v_y, void *grad_t_x, void *grad_v_x,
                             void *stream);

/* Reductions of groups of PCFs (Section 2.1, combinations and reductions;
 * Section 4, Algorithm ReducePair and reduction trees). Group b is PCFs
 * group_offsets_host[b] .. group_offsets_host[b+1]-1 (HOST array, B+1
 * entries, 0 .. n, every group non-empty) and yields one PCF:
 *   PCF_REDUCE_SUM   f_1 + ... + f_m      PCF_REDUCE_MAX / _MIN  pointwise
 *   PCF_REDUCE_MEAN  (f_1 + ... + f_m) / m
 *   PCF_REDUCE_STD   sqrt(sum_i (f_i - mean)^2 / (m - 1)), m >= 2
 * Each group is reduced by a binary tree (neighbours paired level by
 * level, an unpaired last item moving up), and the result keeps a row at
 * t = 0 and wherever the reduced value changes (ReducePair's rule), before
 * the mean or std transformation of the values; a one-PCF group returns its
 * PCF's rows unchanged. Arithmetic in the set's dtype. The tree reads and
 * writes every row of a group once per level (ceil(log2 m) levels); the std
 * evaluates every member at every breakpoint of its group (O(rows x m)).
 * PCF_EINVAL for bad groups or op, PCF_EUNSUPPORTED for 2^31 or more PCFs.
 * Calls: pcf_reduce_workspace_bytes sizes the workspace (device, caller
 * owned); pcf_reduce_rows runs the tree into it, writes the output offsets
 * to offsets_out (device, B+1) and offsets_out_host (host, B+1) and
 * synchronises; pcf_reduce (asynchronous) then writes t_out and v_out
 * (offsets_out_host[B] entries of X's dtype each) from the same workspace,
 * which must be passed unchanged with the same X, groups and op. */
typedef enum {
    PCF_REDUCE_SUM = 0,
    PCF_REDUCE_MEAN = 1,
    PCF_REDUCE_MAX = 2,
    PCF_REDUCE_MIN = 3,
    PCF_REDUCE_STD = 4
} pcf_reduce_op;

pcf_status pcf_reduce_workspace_bytes(const pcf_set *X, int32_t B,
                                      const int64_t *group_offsets_host, pcf_reduce_op op,
                                      size_t *bytes);
pcf_status pcf_reduce_rows(const pcf_set *X, int32_t B, const int64_t *group_offsets_host,
                           pcf_reduce_op op, void *ws, size_t ws_bytes, int64_t *offsets_out,
                           int64_t *offsets_out_host, void *stream);
pcf_status pcf_reduce(const pcf_set *X, int32_t B, const int64_t *group_offsets_host,
                      pcf_reduce_op op, const void *ws, size_t ws_bytes,
                      const int64_t *offsets_out, void *t_out, void *v_out, void *stream);

/* Combinations of two sets index by index (Section 2.1: the induced
 * combination h_*(f, g)(t) = h(f(t), g(t)); Section 4, Algorithm ReducePair):
 * out_i = h_*(x_i, y_i) for X and Y of one dtype and one PCF count n, with
 *   PCF_COMBINE_SUM a + b, _SUB a - b, _MUL a b, _MAX, _MIN, _SQDIFF (a - b)^2.
 * Each result keeps a row at t = 0 and wherever its value changes.
 * PCF_EINVAL for different dtypes or counts or a bad op, PCF_EUNSUPPORTED for
 * 2^30 or more PCFs. Calls as
 * for the reductions: pcf_combine_workspace_bytes; pcf_combine_rows writes
 * offsets_out (device, n+1) and offsets_out_host (host, n+1) and
 * synchronises; pcf_combine (asynchronous) writes t_out and v_out from the
 * same workspace, passed unchanged with the same X, Y and op. */
typedef enum {
    PCF_COMBINE_SUM = 0,
    PCF_COMBINE_SUB = 1,
    PCF_COMBINE_MUL = 2,
    PCF_COMBINE_MAX = 3,
    PCF_COMBINE_MIN = 4,
    PCF_COMBINE_SQDIFF = 5
} pcf_combine_op;

pcf_status pcf_combine_workspace_bytes(const pcf_set *X, const pcf_set *Y, pcf_combine_op op,
                                       size_t *bytes);
pcf_status pcf_combine_rows(const pcf_set *X, const pcf_set *Y, pcf_combine_op op, void *ws,
                            size_t ws_bytes, int64_t *offsets_out, int64_t *offsets_out_host,
                            void *stream);
pcf_status pcf_combine(const pcf_set *X, const pcf_set *Y, pcf_combine_op op, const void *ws,
                       size_t ws_bytes, const int64_t *offsets_out, void *t_out, void *v_out,
                       void *stream);

/* Many independent full matrices in one persistent launch. `all` is one CSR
 * set holding every problem's PCFs; problem b owns PCFs
 * set_offsets_host[b] .. set_offsets_host[b+1]-1 (HOST array, B+1 entries)
 * and its s_b x s_b matrix starts at element out_offsets_host[b] (HOST
 * array, B entries) of `out`, row-major with leading dimension s_b. kind
 * and p as in pcf_pairwise_lp, or PCF_GRAM (p ignored). The tile list
 * covers all problems, ordered by decreasing problem cost. Same errors as
 * pcf_pairwise_lp. */
pcf_status pcf_pairwise_batched(int32_t B, const int64_t *set_offsets_host,
                                const pcf_set *all, pcf_kind kind, double p,
                                void *out, const int64_t *out_offsets_host,
                                void *ws, size_t ws_bytes, uint32_t flags,
                                void *stream);

/* Workspace size for pcf_pairwise_batched. */
pcf_status pcf_batched_workspace_bytes(int32_t B,
                                       const int64_t *set_offsets_host,
                                       const pcf_set *all, size_t *bytes);

/* Data-contract check alone: writes the index of the first PCF that
 * breaks the contract, or -1, to *first_bad (host). ws: at least 256 bytes
 * of device workspace. Synchronises the stream. */
pcf_status pcf_validate(const pcf_set *X, int64_t *first_bad, void *ws,
                        size_t ws_bytes, void *stream);

/* Host-only inspection of the tile plan (no device access): the number of
 * blocks, segments and tiles the library would use for n PCFs with the
 * given host offsets, dtype, window (NULL = full) and backward flag.
 * Used by tests of the planner. */
pcf_status pcf_plan_inspect(int64_t n, const int64_t *offsets_host,
                            pcf_dtype dtype, const pcf_window *w,
                            int backward, int64_t *nblocks, int64_t *nseg,
                            int64_t *ntiles, int32_t *blocks_out,
                            int64_t blocks_cap);

/* Thread-local message describing the last non-OK status. */
const char *pcf_last_error(void);

/* ABI version (bumped on incompatible changes). */
int pcf_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PCF_H */
