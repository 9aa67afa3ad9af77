/*
 * kchol_oracle.c -- plain, slow, CPU reference for the sparse-Cholesky path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the product library: it includes nothing but
 * the C standard library, libquadmath and OpenMP.
 *
 * Everything is FP64 and brute force:
 *   or_maximin        O(N^2) greedy maximin ordering          (Section 2.3)
 *   or_pattern_*      O(N^2) pattern S_rho, max- or min-rule   (Section 2.3; Section 6.2 for min)
 *   or_theta          Matern covariance on S                   (Section 4.4, Matern definition)
 *   or_ichol          right-looking ICHOL(0)                   (Section 2.2, incomplete Cholesky algorithm)
 *   or_solve          L / L^T substitutions                    (Section 1, task (2))
 *   or_llt_pairs      (L L^T)_ab for index pairs               (Section 4.4, error estimate E)
 *   or_frob_error     exact ||L L^T - Theta||_F, ||Theta||_F   (Section 4.4)
 *
 * Built with -ffp-contract=off: no product is fused into a sum unless fma() is
 * written out.  Readings of points where the paper is silent are listed where
 * they are used (first index, ties, pivot rule, zeroed columns in solves).
 */
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2

#define OR_RULE_MAX 0
#define OR_RULE_MIN 1

#define OR_PIVOT_ZERO 0
#define OR_PIVOT_SHIFT 1

/* Euclidean distance, coordinates summed in order t = 0..d-1. */
static double dist(const double *a, const double *b, int d) {
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
        double df = a[t] - b[t];
        s += df * df;
    }
    return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* Maximin ordering, Section 2.3.  Omega = R^d (no boundary), so the first
 * index is arbitrary: we take original index 0 (all distances start at +inf
 * and ties go to the lowest original index, which selects index 0).  Each
 * later step takes the unselected point farthest from the selected set;
 * l[k] is that distance.  perm[k] = original index of the k-th point. */
int or_maximin(const double *x, int64_t n, int32_t d, int32_t *perm, double *l) {
    if (n < 1 || d < 1) return OR_EINVAL;
    double *m = (double *)malloc((size_t)n * sizeof(double));
    unsigned char *sel = (unsigned char *)calloc((size_t)n, 1);
    if (!m || !sel) { free(m); free(sel); return OR_ENOMEM; }
    for (int64_t j = 0; j < n; ++j) m[j] = INFINITY;

    int64_t best = 0; /* argmax of m over unselected points, ties -> lowest index */
    for (int64_t k = 0; k < n; ++k) {
        int64_t i = best;
        perm[k] = (int32_t)i;
        l[k] = m[i];
        sel[i] = 1;
        const double *xi = x + (size_t)i * d;
        int64_t gbest = -1;
        double gval = -1.0;
#pragma omp parallel
        {
            int64_t tb = -1;
            double tv = -1.0;
#pragma omp for schedule(static)
            for (int64_t j = 0; j < n; ++j) {
                if (sel[j]) continue;
                double dj = dist(x + (size_t)j * d, xi, d);
                if (dj < m[j]) m[j] = dj;
                if (m[j] > tv || (m[j] == tv && j < tb)) { tv = m[j]; tb = j; }
            }
#pragma omp critical
            {
                if (tb >= 0 && (tv > gval || (tv == gval && tb < gbest) || gbest < 0)) {
                    gval = tv;
                    gbest = tb;
                }
            }
        }
        best = gbest;
    }
    free(m);
    free(sel);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Sparsity pattern, Section 2.3: (a,b) in S iff dist(x_a,x_b) <= rho*max(l_a,l_b)
 * (max-rule).  The min-rule uses rho*min(l_a,l_b), the pattern given for the
 * reverse-order factor of the inverse in Section 6.2.  Indices are maximin
 * positions; only the lower triangle a >= b is kept, the diagonal always.
 * xh is the point set already gathered into maximin order. */
static int in_pattern(const double *xh, int32_t d, const double *l, double rho, int rule,
                      int64_t a, int64_t b) {
    if (a == b) return 1;
    double la = l[a], lb = l[b];
    double sc = (rule == OR_RULE_MAX) ? (la > lb ? la : lb) : (la < lb ? la : lb);
    double r = dist(xh + (size_t)a * d, xh + (size_t)b * d, d);
    return r <= rho * sc;
}

int or_pattern_count(const double *xh, int64_t n, int32_t d, const double *l, double rho, int32_t rule,
                     int64_t *colptr) {
    if (n < 1 || d < 1 || !(rho > 0.0) || (rule != OR_RULE_MAX && rule != OR_RULE_MIN)) return OR_EINVAL;
    colptr[0] = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < n; ++b) {
        int64_t c = 0;
        for (int64_t a = b; a < n; ++a) c += in_pattern(xh, d, l, rho, rule, a, b);
        colptr[b + 1] = c;
    }
    for (int64_t b = 0; b < n; ++b) colptr[b + 1] += colptr[b];
    return OR_OK;
}

int or_pattern_fill(const double *xh, int64_t n, int32_t d, const double *l, double rho, int32_t rule,
                    const int64_t *colptr, int32_t *rowidx) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < n; ++b) {
        int64_t p = colptr[b];
        for (int64_t a = b; a < n; ++a)
            if (in_pattern(xh, d, l, rho, rule, a, b)) rowidx[p++] = (int32_t)a;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Matern covariance, Section 4.4 definition, at the half-integer smoothness
 * values where it has a closed form (unit variance):
 *   nu = 1/2 : exp(-a),                     a = r/l
 *   nu = 3/2 : (1 + a) exp(-a),             a = sqrt(3) r / l
 *   nu = 5/2 : (1 + a + a^2/3) exp(-a),     a = sqrt(5) r / l
 * The exponential is the correctly rounded one: exp is taken in quad
 * precision and rounded once to double. */
static double cr_exp(double x) { return (double)expq((__float128)x); }

static double matern(double r, int twonu, double ell) {
    if (twonu == 1) {
        double a = r / ell;
        return cr_exp(-a);
    }
    if (twonu == 3) {
        double a = (sqrt(3.0) * r) / ell;
        return (1.0 + a) * cr_exp(-a);
    }
    double a = (sqrt(5.0) * r) / ell;
    return ((1.0 + a) + (a * a) / 3.0) * cr_exp(-a);
}

static int twonu_of(double nu) {
    if (nu == 0.5) return 1;
    if (nu == 1.5) return 3;
    if (nu == 2.5) return 5;
    return 0;
}

int or_matern(const double *r, int64_t m, double nu, double ell, double *out) {
    int tn = twonu_of(nu);
    if (!tn || !(ell > 0.0)) return OR_EINVAL;
    for (int64_t i = 0; i < m; ++i) out[i] = matern(r[i], tn, ell);
    return OR_OK;
}

/* Theta on S in CSC order: theta[e] = G(x_{rowidx[e]}, x_b) for e in column b. */
int or_theta(const double *xh, int64_t n, int32_t d, double nu, double ell, const int64_t *colptr,
             const int32_t *rowidx, double *theta) {
    int tn = twonu_of(nu);
    if (!tn || !(ell > 0.0)) return OR_EINVAL;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < n; ++b)
        for (int64_t e = colptr[b]; e < colptr[b + 1]; ++e) {
            double r = dist(xh + (size_t)rowidx[e] * d, xh + (size_t)b * d, d);
            theta[e] = matern(r, tn, ell);
        }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* ICHOL(0), Section 2.2 (incomplete Cholesky with pattern S), in the paper's
 * right-looking loop order.  For i = 1..N: L_{:i} = A_{:i} / sqrt(A_ii); then for
 * every j > i with (j,i) in S and every k >= j with (k,i),(k,j) in S:
 * A_kj -= L_ki L_ji (the L-form of A_ki A_ji / A_ii), written as one fma.
 * Each entry therefore receives its updates in ascending i.
 * Pivot rule (Section 4.4): a nonpositive pivot zeroes the column, which then
 * contributes no updates (ZERO).  SHIFT instead raises a pivot p <= tau*Theta_ii
 * to tau*Theta_ii and counts it.
 * stats[0] = #nonpositive (zeroed), stats[1] = #shifted, stats[2] = #updates with a
 * nonzero multiplier L_ji (a zeroed column performs none). */
int or_ichol(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *theta, int32_t policy,
             double tau, double *L, int64_t *stats) {
    if (n < 1 || (policy != OR_PIVOT_ZERO && policy != OR_PIVOT_SHIFT)) return OR_EINVAL;
    int64_t *map = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!map) return OR_ENOMEM;
    for (int64_t k = 0; k < n; ++k) map[k] = -1;
    memcpy(L, theta, (size_t)colptr[n] * sizeof(double));
    int64_t nonpos = 0, shifted = 0, updates = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c0 = colptr[i], c1 = colptr[i + 1];
        double p = L[c0]; /* the diagonal is the first entry of the column */
        if (policy == OR_PIVOT_ZERO) {
            if (!(p > 0.0)) {
                for (int64_t e = c0; e < c1; ++e) L[e] = 0.0;
                ++nonpos;
                continue;
            }
        } else {
            double floor_ = tau * theta[c0];
            if (!(p > floor_)) {
                p = floor_;
                ++shifted;
            }
        }
        double s = sqrt(p);
        L[c0] = s;
        for (int64_t e = c0 + 1; e < c1; ++e) L[e] = L[e] / s;
        for (int64_t e = c0; e < c1; ++e) map[rowidx[e]] = e;
        for (int64_t e = c0 + 1; e < c1; ++e) {
            int64_t j = rowidx[e];
            double lji = L[e];
            for (int64_t f = colptr[j]; f < colptr[j + 1]; ++f) {
                int64_t g = map[rowidx[f]];
                if (g >= 0) {
                    L[f] = fma(-L[g], lji, L[f]);
                    if (lji != 0.0) ++updates;
                }
            }
        }
        for (int64_t e = c0; e < c1; ++e) map[rowidx[e]] = -1;
    }
    free(map);
    stats[0] = nonpos;
    stats[1] = shifted;
    stats[2] = updates;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Theta^{-1} b ~ L^{-T} L^{-1} b (Section 1, task (2)) in maximin order.
 * b and y are n x nrhs row-major.  Forward: each y_k takes its updates from
 * columns i < k in ascending i as fma(-L_ki, y_i, .), then is divided by L_kk.
 * Backward: x_j = (y_j - sum_{k in col(j), k>j, ascending} L_kj x_k) / L_jj.
 * A zeroed column (L_jj == 0) gives solution component 0. */
int or_solve(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *L, int32_t nrhs,
             const double *b, double *x) {
    if (n < 1 || nrhs < 1) return OR_EINVAL;
    double *y = (double *)malloc((size_t)n * nrhs * sizeof(double));
    if (!y) return OR_ENOMEM;
    memcpy(y, b, (size_t)n * nrhs * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c0 = colptr[i];
        double lii = L[c0];
        for (int32_t r = 0; r < nrhs; ++r) {
            double *yi = y + (size_t)i * nrhs + r;
            *yi = (lii == 0.0) ? 0.0 : *yi / lii;
        }
        for (int64_t e = c0 + 1; e < colptr[i + 1]; ++e) {
            int64_t k = rowidx[e];
            for (int32_t r = 0; r < nrhs; ++r)
                y[(size_t)k * nrhs + r] = fma(-L[e], y[(size_t)i * nrhs + r], y[(size_t)k * nrhs + r]);
        }
    }
    for (int64_t j = n - 1; j >= 0; --j) {
        int64_t c0 = colptr[j];
        double ljj = L[c0];
        for (int32_t r = 0; r < nrhs; ++r) {
            double acc = y[(size_t)j * nrhs + r];
            for (int64_t e = c0 + 1; e < colptr[j + 1]; ++e)
                acc = fma(-L[e], x[(size_t)rowidx[e] * nrhs + r], acc);
            x[(size_t)j * nrhs + r] = (ljj == 0.0) ? 0.0 : acc / ljj;
        }
    }
    free(y);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Row-major copy of L's structure, for (L L^T)_ab = sum_i L_ai L_bi. */
static int build_rows(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *L,
                      int64_t **rp, int32_t **ci, double **rv) {
    int64_t nnz = colptr[n];
    int64_t *rowptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *col = (int32_t *)malloc((size_t)nnz * sizeof(int32_t));
    double *val = (double *)malloc((size_t)nnz * sizeof(double));
    int64_t *fillp = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!rowptr || !col || !val || !fillp) {
        free(rowptr); free(col); free(val); free(fillp);
        return OR_ENOMEM;
    }
    for (int64_t e = 0; e < nnz; ++e) rowptr[rowidx[e] + 1]++;
    for (int64_t k = 0; k < n; ++k) rowptr[k + 1] += rowptr[k];
    for (int64_t k = 0; k < n; ++k) fillp[k] = rowptr[k];
    for (int64_t j = 0; j < n; ++j)
        for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) {
            int64_t p = fillp[rowidx[e]]++;
            col[p] = (int32_t)j;
            val[p] = L[e];
        }
    free(fillp);
    *rp = rowptr;
    *ci = col;
    *rv = val;
    return OR_OK;
}

static double row_dot(const int64_t *rowptr, const int32_t *col, const double *val, int64_t a, int64_t b) {
    int64_t p = rowptr[a], pe = rowptr[a + 1], q = rowptr[b], qe = rowptr[b + 1];
    double s = 0.0;
    while (p < pe && q < qe) {
        if (col[p] < col[q]) ++p;
        else if (col[p] > col[q]) ++q;
        else { s += val[p] * val[q]; ++p; ++q; }
    }
    return s;
}

/* out[t] = (L L^T)_{a[t], b[t]} (maximin positions). */
int or_llt_pairs(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *L, int64_t npairs,
                 const int64_t *a, const int64_t *b, double *out) {
    int64_t *rowptr; int32_t *col; double *val;
    if (build_rows(n, colptr, rowidx, L, &rowptr, &col, &val)) return OR_ENOMEM;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < npairs; ++t) out[t] = row_dot(rowptr, col, val, a[t], b[t]);
    free(rowptr); free(col); free(val);
    return OR_OK;
}

/* Exact relative Frobenius error over all N^2 pairs (Section 4.4, E without sampling):
 * out[0] = ||L L^T - Theta||_F^2, out[1] = ||Theta||_F^2. */
int or_frob_error(const double *xh, int64_t n, int32_t d, double nu, double ell, const int64_t *colptr,
                  const int32_t *rowidx, const double *L, double *out) {
    int tn = twonu_of(nu);
    if (!tn) return OR_EINVAL;
    int64_t *rowptr; int32_t *col; double *val;
    if (build_rows(n, colptr, rowidx, L, &rowptr, &col, &val)) return OR_ENOMEM;
    double num = 0.0, den = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : num, den)
    for (int64_t a = 0; a < n; ++a)
        for (int64_t b = 0; b < n; ++b) {
            double th = matern(dist(xh + (size_t)a * d, xh + (size_t)b * d, d), tn, ell);
            double df = row_dot(rowptr, col, val, a, b) - th;
            num += df * df;
            den += th * th;
        }
    free(rowptr); free(col); free(val);
    out[0] = num;
    out[1] = den;
    return OR_OK;
}

int or_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* One-by-one versions of the definitions above, for checking samples of a
 * large problem.  xh, l and the pattern are those under test. */

/* out[t] = min_{i < k_t} dist(xh_{k_t}, xh_i): l[k] of the maximin ordering (Section 2.3). */
int or_prefix_min_dist(const double *xh, int32_t d, int64_t m, const int64_t *ks, double *out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < m; ++t) {
        int64_t k = ks[t];
        double best = INFINITY;
        for (int64_t i = 0; i < k; ++i) {
            double r = dist(xh + (size_t)k * d, xh + (size_t)i * d, d);
            if (r < best) best = r;
        }
        out[t] = best;
    }
    return OR_OK;
}

/* Rows of column b of S (Section 2.3), ascending, diagonal first; returns the count
 * (rows must hold n - b entries). */
int64_t or_pattern_column(const double *xh, int64_t n, int32_t d, const double *l, double rho, int32_t rule,
                          int64_t b, int32_t *rows) {
    int64_t c = 0;
    for (int64_t a = b; a < n; ++a)
        if (in_pattern(xh, d, l, rho, rule, a, b)) rows[c++] = (int32_t)a;
    return c;
}

/* Theta_{a_t b_t} (Section 4.4 Matern) for index pairs of the ordered points. */
int or_theta_pairs(const double *xh, int32_t d, double nu, double ell, int64_t m, const int64_t *a,
                   const int64_t *b, double *out) {
    int tn = twonu_of(nu);
    if (!tn || !(ell > 0.0)) return OR_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < m; ++t)
        out[t] = matern(dist(xh + (size_t)a[t] * d, xh + (size_t)b[t] * d, d), tn, ell);
    return OR_OK;
}

/* The first m columns of ICHOL(0) (Section 2.2).  Entries of column j < m are
 * final once columns 0..j-1 have been eliminated, so they can be computed on
 * their own: A_kj = Theta_kj, then for i = 0..j-1 with (j,i),(k,i) in S,
 * ascending, A_kj = fma(-L_ki, L_ji, A_kj) -- the per-entry order of the
 * right-looking algorithm -- followed by the pivot rule and the division.
 * colptr/rowidx: the pattern (CSC); theta: Theta on the first m columns in
 * CSC order (colptr[m] entries); L: output, same layout. */
int or_ichol_leading(int64_t n, const int64_t *colptr, const int32_t *rowidx, int64_t m, const double *theta,
                     int32_t policy, double tau, double *L) {
    if (m < 0 || m > n) return OR_EINVAL;
    int64_t *map = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!map) return OR_ENOMEM;
    for (int64_t k = 0; k < n; ++k) map[k] = -1;
    memcpy(L, theta, (size_t)colptr[m] * sizeof(double));
    for (int64_t j = 0; j < m; ++j) {
        int64_t c0 = colptr[j], c1 = colptr[j + 1];
        for (int64_t e = c0; e < c1; ++e) map[rowidx[e]] = e;
        for (int64_t i = 0; i < j; ++i) {
            int64_t ij = -1; /* position of (j, i) in column i */
            for (int64_t f = colptr[i]; f < colptr[i + 1]; ++f)
                if (rowidx[f] == j) { ij = f; break; }
            if (ij < 0 || L[colptr[i]] == 0.0) continue; /* not a parent, or a zeroed column */
            double lji = L[ij];
            for (int64_t f = ij; f < colptr[i + 1]; ++f) {
                int64_t g = map[rowidx[f]];
                if (g >= 0) L[g] = fma(-L[f], lji, L[g]);
            }
        }
        for (int64_t e = c0; e < c1; ++e) map[rowidx[e]] = -1;
        double p = L[c0];
        if (policy == OR_PIVOT_ZERO) {
            if (!(p > 0.0)) {
                for (int64_t e = c0; e < c1; ++e) L[e] = 0.0;
                continue;
            }
        } else {
            double floor_ = tau * theta[c0];
            if (!(p > floor_)) p = floor_;
        }
        double s = sqrt(p);
        L[c0] = s;
        for (int64_t e = c0 + 1; e < c1; ++e) L[e] = L[e] / s;
    }
    free(map);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Y = Theta X with the dense Matern matrix (Section 4.4), j ascending; X, Y n x nrhs.
 * Used by the conjugate-gradient reference (Sections 4.2-4.3: CG with the sparse
 * factor as preconditioner). */
int or_dense_matvec(const double *x, int64_t n, int32_t d, double nu, double ell, const double *X, int32_t nrhs,
                    double *Y) {
    int tn = twonu_of(nu);
    if (!tn || !(ell > 0.0)) return OR_EINVAL;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t r = 0; r < nrhs; ++r) Y[i * nrhs + r] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double th = matern(dist(x + (size_t)i * d, x + (size_t)j * d, d), tn, ell);
            for (int32_t r = 0; r < nrhs; ++r) Y[i * nrhs + r] += th * X[j * nrhs + r];
        }
    }
    return OR_OK;
}

/* Rows ks of Theta X only (for sampled residuals of large problems). */
int or_dense_matvec_rows(const double *x, int64_t n, int32_t d, double nu, double ell, const double *X,
                         int32_t nrhs, int64_t m, const int64_t *ks, double *Y) {
    int tn = twonu_of(nu);
    if (!tn || !(ell > 0.0)) return OR_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < m; ++t) {
        int64_t i = ks[t];
        for (int32_t r = 0; r < nrhs; ++r) Y[t * nrhs + r] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double th = matern(dist(x + (size_t)i * d, x + (size_t)j * d, d), tn, ell);
            for (int32_t r = 0; r < nrhs; ++r) Y[t * nrhs + r] += th * X[j * nrhs + r];
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Supernodes (the supernodal construction of Section 5's stability analysis),
 * brute force over maximin positions: greedily in maximin order, an unassigned
 * point k starts supernode s and claims every later unassigned point a of the
 * same scale (l_a >= l_k / 2) with dist(x_a, x_k) <= 0.5 * rho * l_k.
 * node[k] receives the supernode of position k; returns the number of supernodes. */
int64_t or_supernodes(const double *xh, int64_t n, int32_t d, const double *l, double rho, int32_t *node) {
    for (int64_t k = 0; k < n; ++k) node[k] = -1;
    int64_t ns = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (node[k] >= 0) continue;
        node[k] = (int32_t)ns;
        double R = 0.5 * rho * l[k], lmin = 0.5 * l[k];
#pragma omp parallel for schedule(static)
        for (int64_t a = k + 1; a < n; ++a)
            if (node[a] < 0 && l[a] >= lmin && dist(xh + (size_t)a * d, xh + (size_t)k * d, d) <= R) node[a] = (int32_t)ns;
        ++ns;
    }
    return ns;
}
