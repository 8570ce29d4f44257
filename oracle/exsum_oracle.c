/*
 * exsum_oracle.c -- CPU oracle for multidimensional included and excluded sums.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke entry point and the benchmark's CPU-baseline leg may load it; the
 * GPU library never links, includes or calls anything here, and nothing here
 * includes or calls the GPU library.
 *
 * Paper: H. Xu, S. Fraser, C. E. Leiserson, "Multidimensional Included and
 * Excluded Sums", SIAM ACDA 2021 (arXiv 2106.00124).
 *
 * What is computed (Sec. 2, "Problem Definitions", Definition "Included and
 * Excluded Sums"): for a d-dimensional tensor A over a monoid (S, op, e) and a
 * box size k, the included sum at x reduces A over the k-box cornered at x,
 * and the excluded sum at x reduces A over every coordinate outside that box.
 *
 * Conventions (the paper uses 1-based coordinates, Sec. 2 "Tensor
 * Preliminaries"; here they are 0-based):
 *   - A is row-major: axis 0 is the paper's dimension 1 (largest stride),
 *     axis d-1 is contiguous.
 *   - box(x) = prod_i [x_i, min(x_i + k_i, n_i)).  Coordinates past the end of
 *     the tensor contribute the identity (Sec. 1, the 2-D definition, and the
 *     clipping rule of the colon notation in Sec. 2).
 *   - Preconditions 1 <= k_i <= n_i (Sec. 1 states k_i <= n_i).
 *
 * Element domains.  Inputs are passed widened:
 *   - floating dtypes (f32, f64) as double; + is evaluated in double (an FP64
 *     reference for f32 inputs), max and min are exact.  Identity: 0 for +,
 *     -inf for max, +inf for min.
 *   - integer dtypes (i32, i64) as int64; + wraps modulo 2^64 (done in uint64)
 *     and, for i32, the result is reduced modulo 2^32 at the end, which equals
 *     the modulo-2^32 sum whatever the order of the additions.  Identity: 0 for
 *     +, the dtype's minimum for max, its maximum for min.
 *
 * Functions:
 *   O1  orc_brute_*       the definition by brute force: O(N^2).
 *   O2  orc_scale_inc_*   included sums as nested window reductions, the
 *                         nesting order of the reduction over a subtensor in
 *                         Sec. 2 (innermost axis first).  O(N sum k).
 *       orc_scale_exc_*   excluded sums: for + as total minus included (the
 *                         box and its complement partition U, and the oracle's
 *                         domains -- doubles, integers mod 2^w -- have an
 *                         inverse); for max and min as a union of half-spaces
 *                         (a point is outside the box iff some coordinate is
 *                         below x_i or at/after x_i + k_i; max and min are
 *                         idempotent, so the overlap of half-spaces does not
 *                         matter).  O(d N).
 *       orc_point_*       one output at a time (sampled checks at full size).
 *   O1/O2 orc_*_vi        the same for a struct element: (value, index)
 *                         pairs ordered by value with the lower index first
 *                         among equal values; max of that total order is
 *                         "argmax", min is "argmin" (commutative monoids, so
 *                         the problem of Sec. 2 is defined for them).
 *   O3  orc_corners2d_*   2-D cross-check after the corners idea (Sec. 1,
 *                         "Corners Algorithm for Strong Excluded Sums"; App. A):
 *                         four disjoint vertex-anchored regions, each an
 *                         orthant reduction.  The region construction is ours.
 *
 * Building with -DORC_MUTANT=<m> plants a known mistake (see the ORC_MUTANT
 * uses below); the test suite builds such variants to show that the pins fail.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif

enum { ORC_F32 = 0, ORC_F64 = 1, ORC_I32 = 2, ORC_I64 = 3 };
enum { ORC_SUM = 0, ORC_MAX = 1, ORC_MIN = 2 };
#define ORC_MAX_RANK 8

/* ------------------------------------------------------------------------ */
/* The monoid (Sec. 1: an associative operator with an identity).           */
/* ------------------------------------------------------------------------ */

static double f_ident(int op) {
    if (op == ORC_SUM) return 0.0;
    return op == ORC_MAX ? -INFINITY : INFINITY;
}
static double f_op(int op, double a, double b) {
    if (op == ORC_SUM) return a + b;
    if (op == ORC_MAX) return a > b ? a : b;
    return a < b ? a : b;
}
static int64_t i_ident(int op, int dtype) {
    if (op == ORC_SUM) return 0;
#if ORC_MUTANT == 6
    if (op == ORC_MIN) return 0; /* planted mistake: wrong identity for min */
#else
    if (op == ORC_MIN) return dtype == ORC_I32 ? (int64_t)INT32_MAX : INT64_MAX;
#endif
#if ORC_MUTANT == 2
    (void)dtype;
    return 0; /* planted mistake: wrong identity for max */
#else
    return dtype == ORC_I32 ? (int64_t)INT32_MIN : INT64_MIN;
#endif
}
static int64_t i_op(int op, int64_t a, int64_t b) {
    if (op == ORC_SUM) return (int64_t)((uint64_t)a + (uint64_t)b); /* wraps */
    if (op == ORC_MAX) return a > b ? a : b;
    return a < b ? a : b;
}
/* Final reduction of an integer + result to the dtype's width (mod 2^32). */
static int64_t i_fix(int op, int dtype, int64_t v) {
#if ORC_MUTANT == 4
    (void)op; (void)dtype;
    return v; /* planted mistake: no wrap to 32 bits */
#else
    if (op == ORC_SUM && dtype == ORC_I32) return (int64_t)(int32_t)(uint32_t)(uint64_t)v;
    return v;
#endif
}

static int check_args(int d, const int64_t *n, const int64_t *k, int64_t *N) {
    if (d < 1 || d > ORC_MAX_RANK) return -1;
    int64_t total = 1;
    for (int i = 0; i < d; ++i) {
        if (n[i] < 1 || k[i] < 1 || k[i] > n[i]) return -1;
        total *= n[i];
    }
    *N = total;
    return 0;
}

/* Flat row-major index -> coordinates. */
static void unflatten(int d, const int64_t *n, int64_t p, int64_t *x) {
    for (int i = d - 1; i >= 0; --i) { x[i] = p % n[i]; p /= n[i]; }
}

/* Is y inside the k-box cornered at x?  (Sec. 2: the box runs from x to
 * x + k along every dimension, half-open.) */
static int in_box(int d, const int64_t *x, const int64_t *k, const int64_t *y) {
    for (int i = 0; i < d; ++i) {
#if ORC_MUTANT == 1
        if (y[i] < x[i] || y[i] > x[i] + k[i]) return 0; /* planted: closed box */
#else
        if (y[i] < x[i] || y[i] >= x[i] + k[i]) return 0;
#endif
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* O1: brute force over every (x, y) pair -- the Definition in Sec. 2.       */
/* inc/exc may be NULL.                                                      */
/* ------------------------------------------------------------------------ */

int orc_brute_f64(int d, const int64_t *n, const int64_t *k, int op,
                  const double *a, double *inc, double *exc) {
    int64_t N;
    if (check_args(d, n, k, &N)) return -1;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < N; ++p) {
        int64_t x[ORC_MAX_RANK], y[ORC_MAX_RANK];
        unflatten(d, n, p, x);
        double si = f_ident(op), se = f_ident(op);
        for (int64_t q = 0; q < N; ++q) {
            unflatten(d, n, q, y);
            if (in_box(d, x, k, y)) si = f_op(op, si, a[q]);
            else                    se = f_op(op, se, a[q]);
        }
        if (inc) inc[p] = si;
        if (exc) exc[p] = se;
    }
    return 0;
}

int orc_brute_i64(int d, const int64_t *n, const int64_t *k, int op, int dtype,
                  const int64_t *a, int64_t *inc, int64_t *exc) {
    int64_t N;
    if (check_args(d, n, k, &N)) return -1;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < N; ++p) {
        int64_t x[ORC_MAX_RANK], y[ORC_MAX_RANK];
        unflatten(d, n, p, x);
        int64_t si = i_ident(op, dtype), se = i_ident(op, dtype);
        for (int64_t q = 0; q < N; ++q) {
            unflatten(d, n, q, y);
            if (in_box(d, x, k, y)) si = i_op(op, si, a[q]);
            else                    se = i_op(op, se, a[q]);
        }
        if (inc) inc[p] = i_fix(op, dtype, si);
        if (exc) exc[p] = i_fix(op, dtype, se);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O2 included: nested window reductions.                                    */
/* The reduction over a subtensor is defined in Sec. 2 as nested reductions, */
/* dimension 1 outermost and dimension d innermost.  Reducing the innermost  */
/* window first for every coordinate, then the next one out, evaluates that  */
/* nesting for all boxes at once: after the pass over axis j,               */
/*   W[x] = op over y_j in [x_j, x_j+k_j), ..., y_{d-1} in [.., ..+k_{d-1})  */
/*          of A[x_0, ..., x_{j-1}, y_j, ..., y_{d-1}].                       */
/* ------------------------------------------------------------------------ */

int orc_scale_inc_f64(int d, const int64_t *n, const int64_t *k, int op,
                      const double *a, double *inc) {
    int64_t N;
    if (check_args(d, n, k, &N)) return -1;
    double *cur = (double *)malloc(sizeof(double) * (size_t)N);
    double *nxt = (double *)malloc(sizeof(double) * (size_t)N);
    if (!cur || !nxt) { free(cur); free(nxt); return -2; }
    memcpy(cur, a, sizeof(double) * (size_t)N);
    int64_t inner = 1;
    for (int j = d - 1; j >= 0; --j) {
        const int64_t len = n[j], stride = inner, outer = N / (len * inner);
        #pragma omp parallel for collapse(2) schedule(static)
        for (int64_t o = 0; o < outer; ++o)
            for (int64_t i = 0; i < inner; ++i) {
                const int64_t base = o * len * stride + i;
                for (int64_t t = 0; t < len; ++t) {
                    double s = f_ident(op);
                    for (int64_t u = t; u < t + k[j] && u < len; ++u)
                        s = f_op(op, s, cur[base + u * stride]);
                    nxt[base + t * stride] = s;
                }
            }
        double *tmp = cur; cur = nxt; nxt = tmp;
        inner *= len;
    }
    memcpy(inc, cur, sizeof(double) * (size_t)N);
    free(cur); free(nxt);
    return 0;
}

int orc_scale_inc_i64(int d, const int64_t *n, const int64_t *k, int op, int dtype,
                      const int64_t *a, int64_t *inc) {
    int64_t N;
    if (check_args(d, n, k, &N)) return -1;
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int64_t *nxt = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    if (!cur || !nxt) { free(cur); free(nxt); return -2; }
    memcpy(cur, a, sizeof(int64_t) * (size_t)N);
    int64_t inner = 1;
    for (int j = d - 1; j >= 0; --j) {
        const int64_t len = n[j], stride = inner, outer = N / (len * inner);
        #pragma omp parallel for collapse(2) schedule(static)
        for (int64_t o = 0; o < outer; ++o)
            for (int64_t i = 0; i < inner; ++i) {
                const int64_t base = o * len * stride + i;
                for (int64_t t = 0; t < len; ++t) {
                    int64_t s = i_ident(op, dtype);
                    for (int64_t u = t; u < t + k[j] && u < len; ++u)
                        s = i_op(op, s, cur[base + u * stride]);
                    nxt[base + t * stride] = s;
                }
            }
        int64_t *tmp = cur; cur = nxt; nxt = tmp;
        inner *= len;
    }
    for (int64_t p = 0; p < N; ++p) inc[p] = i_fix(op, dtype, cur[p]);
    free(cur); free(nxt);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O2 excluded.                                                              */
/* ------------------------------------------------------------------------ */

/* Slab reductions for the half-space cover (op max or min):
 * slab[t] = op of A over y_j == t, pre[j][t] = op over y_j < t (t = 0..n_j),
 * suf[j][t] = op over y_j >= t. */
typedef struct { double *pre[ORC_MAX_RANK], *suf[ORC_MAX_RANK]; } f_cover;
typedef struct { int64_t *pre[ORC_MAX_RANK], *suf[ORC_MAX_RANK]; } i_cover;

static int f_cover_build(int d, const int64_t *n, int64_t N, int op, const double *a,
                         f_cover *c) {
    memset(c, 0, sizeof(*c));
    const double e = f_ident(op);
    for (int j = 0; j < d; ++j) {
        c->pre[j] = (double *)malloc(sizeof(double) * (size_t)(n[j] + 1));
        c->suf[j] = (double *)malloc(sizeof(double) * (size_t)(n[j] + 1));
        if (!c->pre[j] || !c->suf[j]) return -2;
        double *slab = c->suf[j]; /* reuse as scratch */
        for (int64_t t = 0; t <= n[j]; ++t) slab[t] = e;
        int64_t inner = 1;
        for (int m = j + 1; m < d; ++m) inner *= n[m];
        for (int64_t p = 0; p < N; ++p) {
            int64_t t = (p / inner) % n[j];
            slab[t] = f_op(op, slab[t], a[p]);
        }
        c->pre[j][0] = e;
        for (int64_t t = 0; t < n[j]; ++t) c->pre[j][t + 1] = f_op(op, c->pre[j][t], slab[t]);
        /* suffix in place: suf[t] = op over y_j >= t; suf[n_j] = e */
        for (int64_t t = n[j] - 1; t >= 0; --t) slab[t] = f_op(op, slab[t], slab[t + 1]);
    }
    return 0;
}

static int i_cover_build(int d, const int64_t *n, int64_t N, int op, int dtype,
                         const int64_t *a, i_cover *c) {
    memset(c, 0, sizeof(*c));
    const int64_t e = i_ident(op, dtype);
    for (int j = 0; j < d; ++j) {
        c->pre[j] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n[j] + 1));
        c->suf[j] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n[j] + 1));
        if (!c->pre[j] || !c->suf[j]) return -2;
        int64_t *slab = c->suf[j];
        for (int64_t t = 0; t <= n[j]; ++t) slab[t] = e;
        int64_t inner = 1;
        for (int m = j + 1; m < d; ++m) inner *= n[m];
        for (int64_t p = 0; p < N; ++p) {
            int64_t t = (p / inner) % n[j];
            slab[t] = i_op(op, slab[t], a[p]);
        }
        c->pre[j][0] = e;
        for (int64_t t = 0; t < n[j]; ++t) c->pre[j][t + 1] = i_op(op, c->pre[j][t], slab[t]);
        for (int64_t t = n[j] - 1; t >= 0; --t) slab[t] = i_op(op, slab[t], slab[t + 1]);
    }
    return 0;
}

/* Excluded max / min at x: the complement of box(x) is the union over axes j
 * of {y_j < x_j} and {y_j >= x_j + k_j}. */
static double f_cover_at(int d, const int64_t *n, const int64_t *k, int op, const f_cover *c,
                         const int64_t *x) {
    double m = f_ident(op);
    for (int j = 0; j < d; ++j) {
        double lo = c->pre[j][x[j]];
        int64_t hi_start = x[j] + k[j];
        if (hi_start > n[j]) hi_start = n[j];
#if ORC_MUTANT == 5
        double hi = f_ident(op); (void)hi_start; /* planted: suffix half-space dropped */
#else
        double hi = c->suf[j][hi_start];
#endif
        m = f_op(op, m, lo);
        m = f_op(op, m, hi);
    }
    return m;
}

static int64_t i_cover_at(int d, const int64_t *n, const int64_t *k, int op, int dtype,
                          const i_cover *c, const int64_t *x) {
    int64_t m = i_ident(op, dtype);
    for (int j = 0; j < d; ++j) {
        int64_t lo = c->pre[j][x[j]];
        int64_t hi_start = x[j] + k[j];
        if (hi_start > n[j]) hi_start = n[j];
        int64_t hi = c->suf[j][hi_start];
        m = i_op(op, m, lo);
        m = i_op(op, m, hi);
    }
    return m;
}

static void f_cover_free(f_cover *c) {
    for (int j = 0; j < ORC_MAX_RANK; ++j) { free(c->pre[j]); free(c->suf[j]); }
}
static void i_cover_free(i_cover *c) {
    for (int j = 0; j < ORC_MAX_RANK; ++j) { free(c->pre[j]); free(c->suf[j]); }
}

/* inc must hold the included sums (from orc_scale_inc_f64) when op is +. */
/* 1 if k_i = n_i on every axis (the origin's box is the whole tensor). */
static int box_covers_all(int d, const int64_t *n, const int64_t *k) {
    for (int i = 0; i < d; ++i)
        if (k[i] != n[i]) return 0;
    return 1;
}

int orc_scale_exc_f64(int d, const int64_t *n, const int64_t *k, int op,
                      const double *a, const double *inc, double *exc) {
    int64_t N;
    if (check_args(d, n, k, &N)) return -1;
    if (op == ORC_SUM) {
        double total = 0.0;
        for (int64_t p = 0; p < N; ++p) total += a[p];
        #pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < N; ++p) exc[p] = total - inc[p];
        /* With k = n on every axis the box of the origin is the whole tensor:
         * its complement is empty, and the sum over an empty set is the
         * identity (Sec. 2), exactly 0 -- not the rounding residue that
         * total - inc leaves when the two sums run in different orders. */
        if (box_covers_all(d, n, k)) exc[0] = 0.0;
        return 0;
    }
    f_cover c;
    if (f_cover_build(d, n, N, op, a, &c)) { f_cover_free(&c); return -2; }
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        int64_t x[ORC_MAX_RANK];
        unflatten(d, n, p, x);
        exc[p] = f_cover_at(d, n, k, op, &c, x);
    }
    f_cover_free(&c);
    return 0;
}

int orc_scale_exc_i64(int d, const int64_t *n, const int64_t *k, int op, int dtype,
                      const int64_t *a, const int64_t *inc, int64_t *exc) {
    int64_t N;
    if (check_args(d, n, k, &N)) return -1;
    if (op == ORC_SUM) {
        uint64_t total = 0;
        for (int64_t p = 0; p < N; ++p) total += (uint64_t)a[p];
        #pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < N; ++p)
            exc[p] = i_fix(op, dtype, (int64_t)(total - (uint64_t)inc[p]));
        return 0;
    }
    i_cover c;
    if (i_cover_build(d, n, N, op, dtype, a, &c)) { i_cover_free(&c); return -2; }
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        int64_t x[ORC_MAX_RANK];
        unflatten(d, n, p, x);
        exc[p] = i_cover_at(d, n, k, op, dtype, &c, x);
    }
    i_cover_free(&c);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Point oracles: one output per requested flat index.                       */
/* ------------------------------------------------------------------------ */

/* Included sum at each point, reducing the box directly in the nested order
 * of Sec. 2 (axis 0 outermost). */
int orc_point_inc_f64(int d, const int64_t *n, const int64_t *k, int op,
                      const double *a, int64_t npts, const int64_t *pts, double *out) {
    int64_t N;
    if (check_args(d, n, k, &N)) return -1;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < npts; ++s) {
        int64_t x[ORC_MAX_RANK], y[ORC_MAX_RANK], hi[ORC_MAX_RANK];
        unflatten(d, n, pts[s], x);
        for (int i = 0; i < d; ++i) {
            hi[i] = x[i] + k[i] < n[i] ? x[i] + k[i] : n[i];
            y[i] = x[i];
        }
        double acc = f_ident(op);
        for (;;) {
            int64_t q = 0;
            for (int i = 0; i < d; ++i) q = q * n[i] + y[i];
            acc = f_op(op, acc, a[q]);
            int i = d - 1;
            while (i >= 0) {
                if (++y[i] < hi[i]) break;
                y[i] = x[i];
                --i;
            }
            if (i < 0) break;
        }
        out[s] = acc;
    }
    return 0;
}

int orc_point_inc_i64(int d, const int64_t *n, const int64_t *k, int op, int dtype,
                      const int64_t *a, int64_t npts, const int64_t *pts, int64_t *out) {
    int64_t N;
    if (check_args(d, n, k, &N)) return -1;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < npts; ++s) {
        int64_t x[ORC_MAX_RANK], y[ORC_MAX_RANK], hi[ORC_MAX_RANK];
        unflatten(d, n, pts[s], x);
        for (int i = 0; i < d; ++i) {
            hi[i] = x[i] + k[i] < n[i] ? x[i] + k[i] : n[i];
            y[i] = x[i];
        }
        int64_t acc = i_ident(op, dtype);
        for (;;) {
            int64_t q = 0;
#if ORC_MUTANT == 3
            for (int i = d - 1; i >= 0; --i) q = q * n[i] + y[i]; /* planted: axes reversed */
#else
            for (int i = 0; i < d; ++i) q = q * n[i] + y[i];
#endif
            acc = i_op(op, acc, a[q]);
            int i = d - 1;
            while (i >= 0) {
                if (++y[i] < hi[i]) break;
                y[i] = x[i];
                --i;
            }
            if (i < 0) break;
        }
        out[s] = i_fix(op, dtype, acc);
    }
    return 0;
}

/* Excluded sum at each point by the definition: a full pass over the tensor
 * per point (O(N) each).  For a handful of points at full size. */
int orc_point_exc_direct_f64(int d, const int64_t *n, const int64_t *k, int op,
                             const double *a, int64_t npts, const int64_t *pts, double *out) {
    int64_t N;
    if (check_args(d, n, k, &N)) return -1;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < npts; ++s) {
        int64_t x[ORC_MAX_RANK], y[ORC_MAX_RANK];
        unflatten(d, n, pts[s], x);
        for (int i = 0; i < d; ++i) y[i] = 0;
        double acc = f_ident(op);
        for (int64_t q = 0; q < N; ++q) {
            if (!in_box(d, x, k, y)) acc = f_op(op, acc, a[q]);
            int i = d - 1;
            while (i >= 0) { if (++y[i] < n[i]) break; y[i] = 0; --i; }
        }
        out[s] = acc;
    }
    return 0;
}

int orc_point_exc_direct_i64(int d, const int64_t *n, const int64_t *k, int op, int dtype,
                             const int64_t *a, int64_t npts, const int64_t *pts, int64_t *out) {
    int64_t N;
    if (check_args(d, n, k, &N)) return -1;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < npts; ++s) {
        int64_t x[ORC_MAX_RANK], y[ORC_MAX_RANK];
        unflatten(d, n, pts[s], x);
        for (int i = 0; i < d; ++i) y[i] = 0;
        int64_t acc = i_ident(op, dtype);
        for (int64_t q = 0; q < N; ++q) {
            if (!in_box(d, x, k, y)) acc = i_op(op, acc, a[q]);
            int i = d - 1;
            while (i >= 0) { if (++y[i] < n[i]) break; y[i] = 0; --i; }
        }
        out[s] = i_fix(op, dtype, acc);
    }
    return 0;
}

/* Excluded max / min at each point via the half-space cover (O(dN) set-up). */
int orc_point_exc_cover_f64(int d, const int64_t *n, const int64_t *k, int op,
                            const double *a, int64_t npts, const int64_t *pts, double *out) {
    int64_t N;
    if (check_args(d, n, k, &N) || op == ORC_SUM) return -1;
    f_cover c;
    if (f_cover_build(d, n, N, op, a, &c)) { f_cover_free(&c); return -2; }
    for (int64_t s = 0; s < npts; ++s) {
        int64_t x[ORC_MAX_RANK];
        unflatten(d, n, pts[s], x);
        out[s] = f_cover_at(d, n, k, op, &c, x);
    }
    f_cover_free(&c);
    return 0;
}

int orc_point_exc_cover_i64(int d, const int64_t *n, const int64_t *k, int op, int dtype,
                            const int64_t *a, int64_t npts, const int64_t *pts, int64_t *out) {
    int64_t N;
    if (check_args(d, n, k, &N) || op == ORC_SUM) return -1;
    i_cover c;
    if (i_cover_build(d, n, N, op, dtype, a, &c)) { i_cover_free(&c); return -2; }
    for (int64_t s = 0; s < npts; ++s) {
        int64_t x[ORC_MAX_RANK];
        unflatten(d, n, pts[s], x);
        out[s] = i_cover_at(d, n, k, op, dtype, &c, x);
    }
    i_cover_free(&c);
    return 0;
}

/* Threads the parallel loops above use (for reporting the oracle's timing). */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* Reduction of the whole tensor (the identity for an empty tensor cannot
 * occur: N >= 1). */
double orc_total_f64(int64_t N, int op, const double *a) {
    double s = f_ident(op);
    for (int64_t p = 0; p < N; ++p) s = f_op(op, s, a[p]);
    return s;
}
int64_t orc_total_i64(int64_t N, int op, int dtype, const int64_t *a) {
    int64_t s = i_ident(op, dtype);
    for (int64_t p = 0; p < N; ++p) s = i_op(op, s, a[p]);
    return i_fix(op, dtype, s);
}

/* ------------------------------------------------------------------------ */
/* O3: 2-D corners cross-check (strong: no inverse is used).                 */
/* Orthant tables over an n0 x n1 matrix:                                    */
/*   PP[a][b] = op over y0 <= a, y1 <= b     PS[a][b] = op over y0 <= a, y1 >= b */
/*   SS[a][b] = op over y0 >= a, y1 >= b     SP[a][b] = op over y0 >= a, y1 <= b */
/* The complement of the box at x is the disjoint union of                   */
/*   {y0 <  x0,      y1 <  x1+k1}   -> PP[x0-1][min(x1+k1,n1)-1]             */
/*   {y0 <  x0+k0,   y1 >= x1+k1}   -> PS[min(x0+k0,n0)-1][x1+k1]            */
/*   {y0 >= x0+k0,   y1 >= x1}      -> SS[x0+k0][x1]                          */
/*   {y0 >= x0,      y1 <  x1}      -> SP[x0][x1-1]                           */
/* with the identity for an empty region.                                     */
/* ------------------------------------------------------------------------ */

#define IDX(a, b) ((a) * n1 + (b))

int orc_corners2d_f64(int64_t n0, int64_t n1, int64_t k0, int64_t k1, int op,
                      const double *a, double *exc) {
    if (n0 < 1 || n1 < 1 || k0 < 1 || k1 < 1 || k0 > n0 || k1 > n1) return -1;
    size_t sz = sizeof(double) * (size_t)(n0 * n1);
    double *PP = malloc(sz), *PS = malloc(sz), *SS = malloc(sz), *SP = malloc(sz);
    if (!PP || !PS || !SS || !SP) { free(PP); free(PS); free(SS); free(SP); return -2; }
    const double e = f_ident(op);
    for (int64_t i = 0; i < n0; ++i)
        for (int64_t j = 0; j < n1; ++j) {
            double v = a[IDX(i, j)];
            double up = i > 0 ? PP[IDX(i - 1, j)] : e;
            double row = v;
            for (int64_t jj = 0; jj < j; ++jj) row = f_op(op, row, a[IDX(i, jj)]);
            PP[IDX(i, j)] = f_op(op, up, row);
        }
    for (int64_t i = 0; i < n0; ++i)
        for (int64_t j = n1 - 1; j >= 0; --j) {
            double up = i > 0 ? PS[IDX(i - 1, j)] : e;
            double row = a[IDX(i, j)];
            for (int64_t jj = j + 1; jj < n1; ++jj) row = f_op(op, row, a[IDX(i, jj)]);
            PS[IDX(i, j)] = f_op(op, up, row);
        }
    for (int64_t i = n0 - 1; i >= 0; --i)
        for (int64_t j = n1 - 1; j >= 0; --j) {
            double dn = i < n0 - 1 ? SS[IDX(i + 1, j)] : e;
            double row = a[IDX(i, j)];
            for (int64_t jj = j + 1; jj < n1; ++jj) row = f_op(op, row, a[IDX(i, jj)]);
            SS[IDX(i, j)] = f_op(op, dn, row);
        }
    for (int64_t i = n0 - 1; i >= 0; --i)
        for (int64_t j = 0; j < n1; ++j) {
            double dn = i < n0 - 1 ? SP[IDX(i + 1, j)] : e;
            double row = a[IDX(i, j)];
            for (int64_t jj = 0; jj < j; ++jj) row = f_op(op, row, a[IDX(i, jj)]);
            SP[IDX(i, j)] = f_op(op, dn, row);
        }
    for (int64_t x0 = 0; x0 < n0; ++x0)
        for (int64_t x1 = 0; x1 < n1; ++x1) {
            int64_t e0 = x0 + k0 < n0 ? x0 + k0 : n0;   /* end of the box, axis 0 */
            int64_t e1 = x1 + k1 < n1 ? x1 + k1 : n1;   /* end of the box, axis 1 */
            double r = e;
            if (x0 > 0) r = f_op(op, r, PP[IDX(x0 - 1, e1 - 1)]);
            if (e1 < n1) r = f_op(op, r, PS[IDX(e0 - 1, e1)]);
            if (e0 < n0) r = f_op(op, r, SS[IDX(e0, x1)]);
            if (x1 > 0) r = f_op(op, r, SP[IDX(x0, x1 - 1)]);
            exc[IDX(x0, x1)] = r;
        }
    free(PP); free(PS); free(SS); free(SP);
    return 0;
}

int orc_corners2d_i64(int64_t n0, int64_t n1, int64_t k0, int64_t k1, int op, int dtype,
                      const int64_t *a, int64_t *exc) {
    if (n0 < 1 || n1 < 1 || k0 < 1 || k1 < 1 || k0 > n0 || k1 > n1) return -1;
    size_t sz = sizeof(int64_t) * (size_t)(n0 * n1);
    int64_t *PP = malloc(sz), *PS = malloc(sz), *SS = malloc(sz), *SP = malloc(sz);
    if (!PP || !PS || !SS || !SP) { free(PP); free(PS); free(SS); free(SP); return -2; }
    const int64_t e = i_ident(op, dtype);
    for (int64_t i = 0; i < n0; ++i)
        for (int64_t j = 0; j < n1; ++j) {
            int64_t up = i > 0 ? PP[IDX(i - 1, j)] : e;
            int64_t row = a[IDX(i, j)];
            for (int64_t jj = 0; jj < j; ++jj) row = i_op(op, row, a[IDX(i, jj)]);
            PP[IDX(i, j)] = i_op(op, up, row);
        }
    for (int64_t i = 0; i < n0; ++i)
        for (int64_t j = n1 - 1; j >= 0; --j) {
            int64_t up = i > 0 ? PS[IDX(i - 1, j)] : e;
            int64_t row = a[IDX(i, j)];
            for (int64_t jj = j + 1; jj < n1; ++jj) row = i_op(op, row, a[IDX(i, jj)]);
            PS[IDX(i, j)] = i_op(op, up, row);
        }
    for (int64_t i = n0 - 1; i >= 0; --i)
        for (int64_t j = n1 - 1; j >= 0; --j) {
            int64_t dn = i < n0 - 1 ? SS[IDX(i + 1, j)] : e;
            int64_t row = a[IDX(i, j)];
            for (int64_t jj = j + 1; jj < n1; ++jj) row = i_op(op, row, a[IDX(i, jj)]);
            SS[IDX(i, j)] = i_op(op, dn, row);
        }
    for (int64_t i = n0 - 1; i >= 0; --i)
        for (int64_t j = 0; j < n1; ++j) {
            int64_t dn = i < n0 - 1 ? SP[IDX(i + 1, j)] : e;
            int64_t row = a[IDX(i, j)];
            for (int64_t jj = 0; jj < j; ++jj) row = i_op(op, row, a[IDX(i, jj)]);
            SP[IDX(i, j)] = i_op(op, dn, row);
        }
    for (int64_t x0 = 0; x0 < n0; ++x0)
        for (int64_t x1 = 0; x1 < n1; ++x1) {
            int64_t e0 = x0 + k0 < n0 ? x0 + k0 : n0;
            int64_t e1 = x1 + k1 < n1 ? x1 + k1 : n1;
            int64_t r = e;
            if (x0 > 0) r = i_op(op, r, PP[IDX(x0 - 1, e1 - 1)]);
            if (e1 < n1) r = i_op(op, r, PS[IDX(e0 - 1, e1)]);
            if (e0 < n0) r = i_op(op, r, SS[IDX(e0, x1)]);
            if (x1 > 0) r = i_op(op, r, SP[IDX(x0, x1 - 1)]);
            exc[IDX(x0, x1)] = i_fix(op, dtype, r);
        }
    free(PP); free(PS); free(SS); free(SP);
    return 0;
}
#undef IDX

/* ------------------------------------------------------------------------ */
/* A struct monoid: (value, index) pairs.  The order: larger value first for */
/* max (smaller for min); among equal values the lower index comes first.    */
/* max / min of a total order is commutative and associative, with identity  */
/* (-inf, INT32_MAX) for max and (+inf, INT32_MAX) for min: no pair comes     */
/* after it.  The problem of Sec. 2 (a tensor over a monoid) applies as is.  */
/* ------------------------------------------------------------------------ */

typedef struct { double v; int64_t i; } vi_t;

static vi_t vi_ident(int op) {
    vi_t e;
    e.v = op == ORC_MAX ? -INFINITY : INFINITY;
    e.i = INT32_MAX;
    return e;
}
/* Does a come first in the order of op (so that a op b = a)? */
static int vi_first(int op, vi_t a, vi_t b) {
    if (a.v != b.v) return op == ORC_MAX ? a.v > b.v : a.v < b.v;
#if ORC_MUTANT == 7
    return a.i > b.i; /* planted mistake: the higher index wins ties */
#else
    return a.i < b.i;
#endif
}
static vi_t vi_op(int op, vi_t a, vi_t b) { return vi_first(op, a, b) ? a : b; }

static vi_t vi_at(const double *v, const int64_t *idx, int64_t q) {
    vi_t r;
    r.v = v[q];
    r.i = idx[q];
    return r;
}

/* O1 for pairs: every (x, y) pair, inside the box or not (Sec. 2). */
int orc_brute_vi(int d, const int64_t *n, const int64_t *k, int op, const double *v,
                 const int64_t *idx, double *inc_v, int64_t *inc_i, double *exc_v,
                 int64_t *exc_i) {
    int64_t N;
    if (check_args(d, n, k, &N) || op == ORC_SUM) return -1;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < N; ++p) {
        int64_t x[ORC_MAX_RANK], y[ORC_MAX_RANK];
        unflatten(d, n, p, x);
        vi_t si = vi_ident(op), se = vi_ident(op);
        for (int64_t q = 0; q < N; ++q) {
            unflatten(d, n, q, y);
            if (in_box(d, x, k, y)) si = vi_op(op, si, vi_at(v, idx, q));
            else                    se = vi_op(op, se, vi_at(v, idx, q));
        }
        inc_v[p] = si.v; inc_i[p] = si.i;
        exc_v[p] = se.v; exc_i[p] = se.i;
    }
    return 0;
}

/* O2 included for pairs: nested window reductions, innermost axis first
 * (the same nesting as orc_scale_inc_f64). */
int orc_scale_inc_vi(int d, const int64_t *n, const int64_t *k, int op, const double *v,
                     const int64_t *idx, double *inc_v, int64_t *inc_i) {
    int64_t N;
    if (check_args(d, n, k, &N) || op == ORC_SUM) return -1;
    vi_t *cur = (vi_t *)malloc(sizeof(vi_t) * (size_t)N);
    vi_t *nxt = (vi_t *)malloc(sizeof(vi_t) * (size_t)N);
    if (!cur || !nxt) { free(cur); free(nxt); return -2; }
    for (int64_t p = 0; p < N; ++p) cur[p] = vi_at(v, idx, p);
    int64_t inner = 1;
    for (int j = d - 1; j >= 0; --j) {
        const int64_t len = n[j], stride = inner, outer = N / (len * inner);
        #pragma omp parallel for collapse(2) schedule(static)
        for (int64_t o = 0; o < outer; ++o)
            for (int64_t i = 0; i < inner; ++i) {
                const int64_t base = o * len * stride + i;
                for (int64_t t = 0; t < len; ++t) {
                    vi_t s = vi_ident(op);
                    for (int64_t u = t; u < t + k[j] && u < len; ++u)
                        s = vi_op(op, s, cur[base + u * stride]);
                    nxt[base + t * stride] = s;
                }
            }
        vi_t *tmp = cur; cur = nxt; nxt = tmp;
        inner *= len;
    }
    for (int64_t p = 0; p < N; ++p) { inc_v[p] = cur[p].v; inc_i[p] = cur[p].i; }
    free(cur); free(nxt);
    return 0;
}

/* O2 excluded for pairs at the points pts (all N points when pts is NULL):
 * the half-space cover, as for max and min (a cell outside the box lies
 * before or after it along some axis; max / min of a total order is
 * idempotent, so cells in several half-spaces do not matter). */
int orc_exc_cover_vi(int d, const int64_t *n, const int64_t *k, int op, const double *v,
                     const int64_t *idx, int64_t npts, const int64_t *pts, double *exc_v,
                     int64_t *exc_i) {
    int64_t N;
    if (check_args(d, n, k, &N) || op == ORC_SUM) return -1;
    vi_t *pre[ORC_MAX_RANK] = {0}, *suf[ORC_MAX_RANK] = {0};
    int rc = 0;
    const vi_t e = vi_ident(op);
    for (int j = 0; j < d && !rc; ++j) {
        pre[j] = (vi_t *)malloc(sizeof(vi_t) * (size_t)(n[j] + 1));
        suf[j] = (vi_t *)malloc(sizeof(vi_t) * (size_t)(n[j] + 1));
        if (!pre[j] || !suf[j]) { rc = -2; break; }
        /* slab reductions over y_j == t, then prefixes (y_j < t) and
         * suffixes (y_j >= t) of them */
        vi_t *slab = suf[j];
        for (int64_t t = 0; t <= n[j]; ++t) slab[t] = e;
        int64_t inner = 1;
        for (int m = j + 1; m < d; ++m) inner *= n[m];
        for (int64_t p = 0; p < N; ++p) {
            const int64_t t = (p / inner) % n[j];
            slab[t] = vi_op(op, slab[t], vi_at(v, idx, p));
        }
        pre[j][0] = e;
        for (int64_t t = 0; t < n[j]; ++t) pre[j][t + 1] = vi_op(op, pre[j][t], slab[t]);
        for (int64_t t = n[j] - 1; t >= 0; --t) slab[t] = vi_op(op, slab[t], slab[t + 1]);
    }
    if (!rc) {
        const int64_t cnt = pts ? npts : N;
        #pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < cnt; ++s) {
            int64_t x[ORC_MAX_RANK];
            unflatten(d, n, pts ? pts[s] : s, x);
            vi_t m = e;
            for (int j = 0; j < d; ++j) {
                const int64_t hs = x[j] + k[j] < n[j] ? x[j] + k[j] : n[j];
                m = vi_op(op, m, pre[j][x[j]]);
                m = vi_op(op, m, suf[j][hs]);
            }
            exc_v[s] = m.v;
            exc_i[s] = m.i;
        }
    }
    for (int j = 0; j < d; ++j) { free(pre[j]); free(suf[j]); }
    return rc;
}

/* Included pairs at the points pts: a direct reduction over each box. */
int orc_point_inc_vi(int d, const int64_t *n, const int64_t *k, int op, const double *v,
                     const int64_t *idx, int64_t npts, const int64_t *pts, double *inc_v,
                     int64_t *inc_i) {
    int64_t N;
    if (check_args(d, n, k, &N) || op == ORC_SUM) return -1;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < npts; ++s) {
        int64_t x[ORC_MAX_RANK], y[ORC_MAX_RANK], hi[ORC_MAX_RANK];
        unflatten(d, n, pts[s], x);
        for (int i = 0; i < d; ++i) {
            hi[i] = x[i] + k[i] < n[i] ? x[i] + k[i] : n[i];
            y[i] = x[i];
        }
        vi_t acc = vi_ident(op);
        for (;;) {
            int64_t q = 0;
            for (int i = 0; i < d; ++i) q = q * n[i] + y[i];
            acc = vi_op(op, acc, vi_at(v, idx, q));
            int i = d - 1;
            while (i >= 0) {
                if (++y[i] < hi[i]) break;
                y[i] = x[i];
                --i;
            }
            if (i < 0) break;
        }
        inc_v[s] = acc.v;
        inc_i[s] = acc.i;
    }
    return 0;
}

