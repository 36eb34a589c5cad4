/*
 * pcf_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU reference for the pairwise
 * integrated-combination matrices of piecewise constant functions (PCFs).
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the GPU library never links, calls or reads it,
 * and the two share no source.
 *
 * What it computes (paper, Section 3, Eq. "simpleint" and Section 2.2,
 * "Functionals"):
 *
 *   A PCF f is given by n >= 1 rows (t_k, v_k), k = 0..n-1, with
 *   0 = t_0 < t_1 < ... < t_{n-1}; f(x) = v_k on [t_k, t_{k+1}) and
 *   f(x) = v_{n-1} on [t_{n-1}, inf)                      (Section 2).
 *   For two PCFs f, g let s_0 < s_1 < ... < s_{m-1} be the union of their
 *   breakpoints -- a common discretization (Section 2, minimal common
 *   refinement). Then (Eq. simpleint)
 *
 *       I_h(f, g) = sum_{r=0}^{m-2} h(f(s_r), g(s_r)) * (s_{r+1} - s_r)
 *
 *   plus the unbounded last cell [s_{m-1}, inf), which contributes 0 when
 *   h(f(s_{m-1}), g(s_{m-1})) == 0 (the eventually-zero case the paper
 *   assumes) and an infinity of the sign of h otherwise.
 *
 *   Combination integrals F = r(I_h) (Section 2.2):
 *     ORC_LP      h = |a-b|^p, r(x) = x^(1/p)   (L_p distance)
 *     ORC_LP_POW  h = |a-b|^p, r(x) = x        (d_p^p, no root)
 *     ORC_GRAM    h = a*b,     r(x) = x        (L_2 inner product)
 *
 * The oracle forms the union grid explicitly (a textbook merge of two
 * sorted lists, duplicates dropped), evaluates f and g on it from the
 * definition of a PCF, and sums the cells left to right with one rounding
 * per multiply and per add (build with -ffp-contract=off, no fast-math).
 *
 * Single-PCF functionals F(f) = r(int_a^b h(f)) (Section 3.2) follow
 * Algorithm IterateSegments: see orc_single below. Pair integrals over a
 * range [a, b) clip every cell to it (integral_ab); a time-dependent
 * h = h0 w(t) adds H(r) - H(l) per cell with H = h0 W (integral_w).
 *
 * The adjoint (derivatives of F with respect to the values v_k and the
 * breakpoint times t_k, k >= 1) is not in the paper. Its reading:
 *   dI/dv_f[k] = sum over cells r where f takes its k-th value of
 *                (dh/da)(f(s_r), g(s_r)) * (s_{r+1} - s_r)
 *   dI/dt_f[k] = h(v_f[k-1], g(t_k)) - h(v_f[k], g(t_k))   for k >= 1,
 *                with g(t_k) the value of g just after t_k for the right
 *                derivative and just before t_k for the left derivative;
 *                where g also breaks at t_k the two differ and the mean of
 *                both one-sided derivatives is used.
 *   t_0 and the last value are fixed by the PCF contract: gradient 0.
 *   dF/dI = (1/p) I^(1/p - 1) for ORC_LP (0 when I == 0), 1 otherwise.
 *   dh/da for |a-b|^p: p |a-b|^(p-1) sign(a-b) with sign(0) = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_LP = 0, ORC_LP_POW = 1, ORC_GRAM = 2 };

/* h(a, b) of the combination integral (Section 2.2). p == 1 and p == 2
 * are written without pow so that they are exact products. */
static double h_val(int kind, double p, double a, double b)
{
    if (kind == ORC_GRAM)
        return a * b;
    double d = fabs(a - b);
    if (p == 1.0)
        return d;
    if (p == 2.0)
        return d * d;
    return pow(d, p);
}

/* dh/da (the first argument). h is symmetric for every kind, so dh/db at
 * (a, b) equals dh/da at (b, a). */
static double dh_da(int kind, double p, double a, double b)
{
    if (kind == ORC_GRAM)
        return b;
    double d = a - b;
    double s = (d > 0.0) ? 1.0 : ((d < 0.0) ? -1.0 : 0.0);
    if (p == 1.0)
        return s;
    if (p == 2.0)
        return 2.0 * d;
    return p * pow(fabs(d), p - 1.0) * s;
}

/* The PCF contract (Section 2 and the user guide): at least one row,
 * t_0 = 0, strictly increasing finite times, finite values. Returns 1 when
 * it holds. (A nonzero last value is allowed here: the tail rule above
 * gives it a meaning.) */
static int pcf_ok(const double *t, const double *v, int64_t n)
{
    if (n < 1 || t[0] != 0.0)
        return 0;
    for (int64_t k = 0; k < n; ++k) {
        if (!isfinite(t[k]) || !isfinite(v[k]))
            return 0;
        if (k > 0 && !(t[k] > t[k - 1]))
            return 0;
    }
    return 1;
}

/* Union of two sorted breakpoint lists, equal times kept once. s must hold
 * nf + ng doubles. Returns the number of grid points m. */
static int64_t union_grid(const double *tf, int64_t nf, const double *tg,
                          int64_t ng, double *s)
{
    int64_t i = 0, j = 0, m = 0;
    while (i < nf || j < ng) {
        double x;
        if (j >= ng || (i < nf && tf[i] <= tg[j]))
            x = tf[i++];
        else
            x = tg[j++];
        if (m == 0 || x != s[m - 1])
            s[m++] = x;
    }
    return m;
}

/* Index of the row of a PCF whose piece contains x: max{k : t_k <= x}
 * (x >= t_0 = 0). Plain binary search. */
static int64_t piece_at(const double *t, int64_t n, double x)
{
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo + 1) / 2;
        if (t[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

/* Index of the piece just before x: max{k : t_k < x}, for x > 0. */
static int64_t piece_before(const double *t, int64_t n, double x)
{
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo + 1) / 2;
        if (t[mid] < x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

/* I_h(f, g) by Eq. simpleint over the union grid, restricted to the
 * integration range [a, b) of Section 2.2 (0 <= a < b <= inf): each cell
 * [s_r, s_{r+1}) counts with its part inside [a, b). scratch holds nf + ng
 * doubles. *abs_out (optional) receives sum |h| * width, the scale used for
 * cancellation-aware tolerances. Returns NaN when either PCF breaks the
 * contract. */
static double integral_ab(int kind, double p, double a, double b, const double *tf,
                          const double *vf, int64_t nf, const double *tg,
                          const double *vg, int64_t ng, double *scratch,
                          double *abs_out)
{
    if (!pcf_ok(tf, vf, nf) || !pcf_ok(tg, vg, ng)) {
        if (abs_out)
            *abs_out = NAN;
        return NAN;
    }
    int64_t m = union_grid(tf, nf, tg, ng, scratch);
    double acc = 0.0, acc_abs = 0.0;
    int64_t kf = 0, kg = 0;
    for (int64_t r = 0; r < m; ++r) {
        double x = scratch[r];
        /* f(x), g(x): the piece containing x (pointers only move right
         * because the grid is increasing). */
        while (kf + 1 < nf && tf[kf + 1] <= x)
            ++kf;
        while (kg + 1 < ng && tg[kg + 1] <= x)
            ++kg;
        double hv = h_val(kind, p, vf[kf], vg[kg]);
        /* the cell's part inside [a, b) */
        double l = x < a ? a : x;
        if (r + 1 < m) {
            double rr = scratch[r + 1] > b ? b : scratch[r + 1];
            double w = rr > l ? rr - l : 0.0;
            double c = hv * w;
            acc = acc + c;
            acc_abs = acc_abs + fabs(c);
        } else if (isinf(b)) {
            /* unbounded last cell */
            if (hv != 0.0) {
                acc = acc + (hv > 0.0 ? INFINITY : -INFINITY);
                acc_abs = INFINITY;
            }
        } else {
            double w = b > l ? b - l : 0.0;
            double c = hv * w;
            acc = acc + c;
            acc_abs = acc_abs + fabs(c);
        }
    }
    if (abs_out)
        *abs_out = acc_abs;
    return acc;
}

static double integral(int kind, double p, const double *tf, const double *vf,
                       int64_t nf, const double *tg, const double *vg,
                       int64_t ng, double *scratch, double *abs_out)
{
    return integral_ab(kind, p, 0.0, INFINITY, tf, vf, nf, tg, vg, ng, scratch,
                       abs_out);
}

static double finish(int kind, double p, double I)
{
    if (kind != ORC_LP)
        return I;
    if (p == 1.0)
        return I;
    if (p == 2.0)
        return sqrt(I);
    return pow(I, 1.0 / p);
}

/* ---------------------------------------------------------------------- */
/* Exported entry points (ctypes).                                          */

/* One combination integral F(f, g). scratch: nf + ng doubles or NULL. */
double orc_pair(int kind, double p, const double *tf, const double *vf,
                int64_t nf, const double *tg, const double *vg, int64_t ng,
                double *abs_out)
{
    double *s = (double *)malloc(sizeof(double) * (size_t)(nf + ng + 1));
    if (!s)
        return NAN;
    double I = integral(kind, p, tf, vf, nf, tg, vg, ng, s, abs_out);
    free(s);
    return finish(kind, p, I);
}

/* F for a list of ordered pairs (I[k], J[k]) of a CSR set: PCF i has rows
 * offsets[i] .. offsets[i+1]-1 of t and v. out[k] = F(f_I[k], f_J[k]),
 * abs_out[k] (optional) = sum |h| * width. Returns 0, or -1 on bad
 * arguments. */
int orc_entries(int kind, double p, int64_t n_pcf, const int64_t *offsets,
                const double *t, const double *v, int64_t npairs,
                const int64_t *I, const int64_t *J, double *out,
                double *abs_out)
{
    int64_t nmax = 0;
    for (int64_t i = 0; i < n_pcf; ++i) {
        int64_t n = offsets[i + 1] - offsets[i];
        if (n > nmax)
            nmax = n;
    }
    double *s = (double *)malloc(sizeof(double) * (size_t)(2 * nmax + 1));
    if (!s)
        return -1;
    for (int64_t k = 0; k < npairs; ++k) {
        int64_t a = I[k], b = J[k];
        if (a < 0 || b < 0 || a >= n_pcf || b >= n_pcf) {
            free(s);
            return -1;
        }
        const int64_t oa = offsets[a], ob = offsets[b];
        double ab = 0.0;
        double Iv = integral(kind, p, t + oa, v + oa, offsets[a + 1] - oa,
                             t + ob, v + ob, offsets[b + 1] - ob, s, &ab);
        out[k] = finish(kind, p, Iv);
        if (abs_out)
            abs_out[k] = ab;
    }
    free(s);
    return 0;
}

/* As orc_entries over the integration range [a, b) (0 <= a < b <= inf). */
int orc_entries_ab(int kind, double p, double a, double b, int64_t n_pcf,
                   const int64_t *offsets, const double *t, const double *v,
                   int64_t npairs, const int64_t *I, const int64_t *J, double *out,
                   double *abs_out)
{
    if (!(a >= 0.0) || !(b > a))
        return -1;
    int64_t nmax = 0;
    for (int64_t i = 0; i < n_pcf; ++i) {
        int64_t n = offsets[i + 1] - offsets[i];
        if (n > nmax)
            nmax = n;
    }
    double *s = (double *)malloc(sizeof(double) * (size_t)(2 * nmax + 1));
    if (!s)
        return -1;
    for (int64_t k = 0; k < npairs; ++k) {
        int64_t i = I[k], j = J[k];
        if (i < 0 || j < 0 || i >= n_pcf || j >= n_pcf) {
            free(s);
            return -1;
        }
        const int64_t oi = offsets[i], oj = offsets[j];
        double ab = 0.0;
        double Iv = integral_ab(kind, p, a, b, t + oi, v + oi, offsets[i + 1] - oi,
                                t + oj, v + oj, offsets[j + 1] - oj, s, &ab);
        out[k] = finish(kind, p, Iv);
        if (abs_out)
            abs_out[k] = ab;
    }
    free(s);
    return 0;
}

/* Time-dependent combinations (Section 2.2, weighted L_p and weighted
 * inner product; Section 3, the time-dependent h with a known antiderivative
 * H in t). The weight w >= 0 multiplies a time-independent h:
 * h(a, b, t) = h0(a, b) w(t), so H(a, b, t) = h0(a, b) W(t) with
 * W(t) = int_0^t w. Two weight families with closed-form W:
 *   ORC_W_EXP  w(t) = exp(-c t), c > 0:   W(t) = (1 - exp(-c t)) / c
 *   ORC_W_POW  w(t) = t^c, c > -1:        W(t) = t^(c+1) / (c+1)      */
#define ORC_W_EXP 1
#define ORC_W_POW 2

static double w_anti(int wk, double c, double t)
{
    if (wk == ORC_W_EXP)
        return isinf(t) ? 1.0 / c : -expm1(-c * t) / c;
    return isinf(t) ? INFINITY : pow(t, c + 1.0) / (c + 1.0);
}

/* I = sum over the cells [l, r) of the common refinement, clipped to
 * [a, b), of H(f(l), g(l), r) - H(f(l), g(l), l) (Section 3). *abs_out
 * (optional) receives sum |h0| (|W(r)| + |W(l)|): the magnitudes of the
 * terms the sum adds, the scale of its rounding error. */
static double integral_w(int kind, double p, int wk, double c, double a, double b,
                         const double *tf, const double *vf, int64_t nf,
                         const double *tg, const double *vg, int64_t ng,
                         double *scratch, double *abs_out)
{
    if (!pcf_ok(tf, vf, nf) || !pcf_ok(tg, vg, ng)) {
        if (abs_out)
            *abs_out = NAN;
        return NAN;
    }
    int64_t m = union_grid(tf, nf, tg, ng, scratch);
    double acc = 0.0, acc_abs = 0.0;
    int64_t kf = 0, kg = 0;
    for (int64_t r = 0; r < m; ++r) {
        double x = scratch[r];
        while (kf + 1 < nf && tf[kf + 1] <= x)
            ++kf;
        while (kg + 1 < ng && tg[kg + 1] <= x)
            ++kg;
        double h0 = h_val(kind, p, vf[kf], vg[kg]);
        double l = x < a ? a : x;
        double rr = r + 1 < m ? scratch[r + 1] : INFINITY;
        if (rr > b)
            rr = b;
        if (!(rr > l) || h0 == 0.0)
            continue; /* empty cell, or a zero integrand (the unbounded tail) */
        double Hr = h0 * w_anti(wk, c, rr), Hl = h0 * w_anti(wk, c, l);
        acc = acc + (Hr - Hl);
        acc_abs = acc_abs + fabs(Hr) + fabs(Hl);
    }
    if (abs_out)
        *abs_out = acc_abs;
    return acc;
}

/* As orc_entries_ab with the weight (wk, c): F = r(I) of integral_w.
 * Returns -1 on bad indices, bounds or weight parameters. */
int orc_entries_w(int kind, double p, int wk, double c, double a, double b,
                  int64_t n_pcf, const int64_t *offsets, const double *t,
                  const double *v, int64_t npairs, const int64_t *I,
                  const int64_t *J, double *out, double *abs_out)
{
    if (!(a >= 0.0) || !(b > a))
        return -1;
    if (!((wk == ORC_W_EXP && c > 0.0 && isfinite(c)) ||
          (wk == ORC_W_POW && c > -1.0 && isfinite(c))))
        return -1;
    int64_t nmax = 0;
    for (int64_t i = 0; i < n_pcf; ++i) {
        int64_t n = offsets[i + 1] - offsets[i];
        if (n > nmax)
            nmax = n;
    }
    double *s = (double *)malloc(sizeof(double) * (size_t)(2 * nmax + 1));
    if (!s)
        return -1;
    for (int64_t k = 0; k < npairs; ++k) {
        int64_t i = I[k], j = J[k];
        if (i < 0 || j < 0 || i >= n_pcf || j >= n_pcf) {
            free(s);
            return -1;
        }
        const int64_t oi = offsets[i], oj = offsets[j];
        double ab = 0.0;
        double Iv = integral_w(kind, p, wk, c, a, b, t + oi, v + oi, offsets[i + 1] - oi,
                               t + oj, v + oj, offsets[j + 1] - oj, s, &ab);
        out[k] = finish(kind, p, Iv);
        if (abs_out)
            abs_out[k] = ab;
    }
    free(s);
    return 0;
}

/* Full M x M matrix F(C) (Section 3.1): every entry computed on its own,
 * symmetry not assumed. out is row-major with leading dimension M. */
int orc_matrix(int kind, double p, int64_t n_pcf, const int64_t *offsets,
               const double *t, const double *v, double *out)
{
    for (int64_t i = 0; i < n_pcf; ++i) {
        int64_t *J = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_pcf);
        int64_t *I = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_pcf);
        if (!I || !J) {
            free(I);
            free(J);
            return -1;
        }
        for (int64_t j = 0; j < n_pcf; ++j) {
            I[j] = i;
            J[j] = j;
        }
        int rc = orc_entries(kind, p, n_pcf, offsets, t, v, n_pcf, I, J,
                             out + i * n_pcf, NULL);
        free(I);
        free(J);
        if (rc)
            return rc;
    }
    return 0;
}

/* Adds w * dI/d(theta_f) into (gt, gv) for one side f of the pair (f, g):
 * the values v_f[k] and the times t_f[k], k >= 1, following the reading in
 * the header comment. */
static void side_grad(int kind, double p, const double *tf, const double *vf,
                      int64_t nf, const double *tg, const double *vg,
                      int64_t ng, double w, double *gt, double *gv,
                      double *scratch)
{
    int64_t m = union_grid(tf, nf, tg, ng, scratch);
    /* values: cell contributions */
    for (int64_t r = 0; r + 1 < m; ++r) {
        double x = scratch[r];
        int64_t kf = piece_at(tf, nf, x);
        int64_t kg = piece_at(tg, ng, x);
        double width = scratch[r + 1] - x;
        gv[kf] += w * dh_da(kind, p, vf[kf], vg[kg]) * width;
    }
    /* times: each breakpoint t_k, k >= 1, moves the boundary between the
     * pieces k-1 and k of f */
    for (int64_t k = 1; k < nf; ++k) {
        double x = tf[k];
        double g_right = vg[piece_at(tg, ng, x)];
        double g_left = vg[piece_before(tg, ng, x)];
        double d_right = h_val(kind, p, vf[k - 1], g_right) -
                         h_val(kind, p, vf[k], g_right);
        double d_left = h_val(kind, p, vf[k - 1], g_left) -
                        h_val(kind, p, vf[k], g_left);
        gt[k] += w * 0.5 * (d_right + d_left);
    }
    /* the last value and t_0 are fixed parameters */
    gv[nf - 1] = 0.0;
    gt[0] = 0.0;
}

/* Gradient of L = sum_{i,j} G[i*M + j] * F(f_i, f_j) over all ordered
 * pairs, with respect to t and v of every PCF (CSR layout, same as the
 * input). gt and gv are overwritten. Returns 0, or -1 on failure. */
int orc_backward(int kind, double p, int64_t n_pcf, const int64_t *offsets,
                 const double *t, const double *v, const double *G,
                 double *gt, double *gv)
{
    int64_t P = offsets[n_pcf]; /* t, v, gt, gv are indexed from 0 */
    memset(gt, 0, sizeof(double) * (size_t)P);
    memset(gv, 0, sizeof(double) * (size_t)P);
    int64_t nmax = 0;
    for (int64_t i = 0; i < n_pcf; ++i) {
        int64_t n = offsets[i + 1] - offsets[i];
        if (n > nmax)
            nmax = n;
    }
    double *s = (double *)malloc(sizeof(double) * (size_t)(2 * nmax + 1));
    if (!s)
        return -1;
    for (int64_t i = 0; i < n_pcf; ++i) {
        for (int64_t j = 0; j < n_pcf; ++j) {
            double gij = G[i * n_pcf + j];
            if (gij == 0.0)
                continue;
            const int64_t oi = offsets[i], oj = offsets[j];
            const int64_t ni = offsets[i + 1] - oi, nj = offsets[j + 1] - oj;
            double chain = 1.0;
            if (kind == ORC_LP && p != 1.0) {
                double I = integral(kind, p, t + oi, v + oi, ni, t + oj,
                                    v + oj, nj, s, NULL);
                chain = (I > 0.0) ? (1.0 / p) * pow(I, 1.0 / p - 1.0) : 0.0;
            }
            double w = gij * chain;
            /* F depends on f_i through its first argument and on f_j
             * through its second; h is symmetric, so the second argument's
             * derivative is the first-argument formula with roles swapped.
             * For i == j both contributions land on the same PCF. */
            side_grad(kind, p, t + oi, v + oi, ni, t + oj, v + oj, nj, w,
                      gt + oi, gv + oi, s);
            side_grad(kind, p, t + oj, v + oj, nj, t + oi, v + oi, ni, w,
                      gt + oj, gv + oj, s);
        }
    }
    free(s);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Single-PCF functionals (Section 3.2, "PCF integrals"):                   */
/*     F(f) = r( int_a^b h(f(t)) dt ),  0 <= a < b <= inf,                   */
/* by segment iteration (Algorithm IterateSegments): start at t = a in the   */
/* piece that contains a; each later breakpoint t_i closes the segment       */
/* [t, min(t_i, b)) of the current value, the walk stops once t_i >= b; the  */
/* last segment runs from the current left end to b. Each segment (l, r, v)  */
/* adds (r - l) h(v), left to right. With b = inf the last segment adds 0    */
/* when h(v) = 0 and an infinity of the sign of h(v) otherwise.              */
/*   ORC_S_INTEGRAL  h(v) = v                                               */
/*   ORC_S_NORM      h(v) = |v|^p, r(x) = x^(1/p)                           */
/*   ORC_S_NORM_POW  h(v) = |v|^p, r(x) = x                                 */
/*   ORC_S_NORM_INF  sup |f| over [a, b): the largest |v| of the segments    */
enum { ORC_S_INTEGRAL = 0, ORC_S_NORM = 1, ORC_S_NORM_POW = 2, ORC_S_NORM_INF = 3 };

static double h_single(int kind, double p, double v)
{
    if (kind == ORC_S_INTEGRAL)
        return v;
    double a = fabs(v);
    if (p == 1.0)
        return a;
    if (p == 2.0)
        return a * a;
    return pow(a, p);
}

static double segment_sum(int kind, double p, double a, double b, const double *t,
                          const double *v, int64_t n, double *abs_out)
{
    double acc = 0.0, acc_abs = 0.0;
    double l = a;
    int64_t k = piece_at(t, n, a);
    double val = v[k];
    int done = 0;
    for (int64_t i = k + 1; i < n; ++i) {
        double r = t[i] < b ? t[i] : b;
        double c = (r - l) * h_single(kind, p, val);
        acc = acc + c;
        acc_abs = acc_abs + fabs(c);
        if (t[i] >= b) {
            done = 1;
            break;
        }
        l = t[i];
        val = v[i];
    }
    if (!done) {
        double hv = h_single(kind, p, val);
        if (isinf(b)) {
            if (hv != 0.0) {
                acc = acc + (hv > 0.0 ? INFINITY : -INFINITY);
                acc_abs = INFINITY;
            }
        } else {
            double c = (b - l) * hv;
            acc = acc + c;
            acc_abs = acc_abs + fabs(c);
        }
    }
    if (abs_out)
        *abs_out = acc_abs;
    return acc;
}

/* sup over [a, b) of |f|: Algorithm IterateSegments, keeping the largest
 * |v| of the segments it lists (each has r > l). */
static double segment_max(double a, double b, const double *t, const double *v, int64_t n)
{
    double l = a;
    int64_t k = piece_at(t, n, a);
    double val = v[k];
    double m = 0.0;
    for (int64_t i = k + 1; i < n; ++i) {
        double r = t[i] < b ? t[i] : b;
        if (r > l && fabs(val) > m)
            m = fabs(val);
        if (t[i] >= b)
            return m;
        l = t[i];
        val = v[i];
    }
    if (b > l && fabs(val) > m)
        m = fabs(val);
    return m;
}

/* F(f_i) for every PCF of a CSR set; abs_out[i] (optional) = sum over
 * segments of |h| * width. Returns 0, or -1 on bad arguments. */
int orc_single(int kind, double p, double a, double b, int64_t n_pcf,
               const int64_t *offsets, const double *t, const double *v,
               double *out, double *abs_out)
{
    if (!(a >= 0.0) || !(b > a))
        return -1;
    for (int64_t i = 0; i < n_pcf; ++i) {
        const int64_t o = offsets[i], n = offsets[i + 1] - offsets[i];
        double ab = 0.0;
        double I;
        if (n < 1 || !pcf_ok(t + o, v + o, n)) {
            I = NAN;
            ab = NAN;
        } else if (kind == ORC_S_NORM_INF) {
            I = segment_max(a, b, t + o, v + o, n);
            ab = I;
        } else {
            I = segment_sum(kind, p, a, b, t + o, v + o, n, &ab);
        }
        if (kind == ORC_S_NORM && p != 1.0)
            I = p == 2.0 ? sqrt(I) : pow(I, 1.0 / p);
        out[i] = I;
        if (abs_out)
            abs_out[i] = ab;
    }
    return 0;
}

int orc_abi_version(void) { return 1; }
