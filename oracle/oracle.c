/*
 * Oracle for the diagonal-scaling preprocessing of the optimal assignment
 * problem (Sharify, Gaubert, Grigori, "Solution of the optimal assignment
 * problem by diagonal scaling algorithms", arXiv:1104.3830).
 *
 * TEST INFRASTRUCTURE ONLY. This file is a plain, slow, FP64 CPU statement of
 * what the GPU library computes. Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code with the HIP library.
 *
 * Notation follows the paper. The input is the log-weight matrix
 * b_ij = log a_ij (row-major, n x n, -INFINITY where a_ij = 0). The scalings
 * are held as ubar = p^-1 log u and vbar = p^-1 log v (Section 4.1.2), so the
 * scaled matrix is x_ij = exp(p (b_ij + ubar_i + vbar_j)).
 *
 * Parallelism: OpenMP over independent rows or columns only; every sum is
 * taken by one thread in index order, so results do not depend on the thread
 * count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define B_(i, j) B[(size_t)(i) * (size_t)n + (size_t)(j)]
#define R_(i, j) B[(size_t)(i) * (size_t)cols + (size_t)(j)]

/* Row step of the logarithmic p-Sinkhorn iteration (Section 4.1.2):
 *   ubar_i = -max_j(b_ij + vbar_j) - p^-1 log sum_j exp(p xhat_ij),
 *   xhat_ij = b_ij + vbar_j - max_j(b_ij + vbar_j).
 * This is u = I(A^(p) v) of the u/v form of Sinkhorn (eq. dad2) in log
 * coordinates, for a block of `rows` rows of a matrix with `cols` columns
 * (each row is independent). Returns the number of rows with no finite entry
 * (then ubar_i = +inf). */
int or_row_step(int rows, int cols, double p, const double *B, const double *vbar, double *ubar)
{
    int bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(static) if (rows >= 128)
    for (int i = 0; i < rows; ++i) {
        double mx = -INFINITY;
        for (int j = 0; j < cols; ++j) {
            double y = R_(i, j) + vbar[j];
            if (y > mx) mx = y;
        }
        if (mx == -INFINITY) {
            ubar[i] = INFINITY;
            bad += 1;
            continue;
        }
        double s = 0.0;
        for (int j = 0; j < cols; ++j) {
            double y = R_(i, j) + vbar[j];
            if (y != -INFINITY) s += exp(p * (y - mx));
        }
        ubar[i] = -mx - log(s) / p;
    }
    return bad;
}

/* Column step (Section 4.1.2; v = I(A^(p)T u), eq. dad3), for a block of
 * `cols` columns over `rows` rows (each column is independent):
 *   vbar_j = -max_i(b_ij + ubar_i) - p^-1 log sum_i exp(p yhat_ij). */
int or_col_step(int rows, int cols, double p, const double *B, const double *ubar, double *vbar)
{
    int bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(static) if (cols >= 128)
    for (int j = 0; j < cols; ++j) {
        double mx = -INFINITY;
        for (int i = 0; i < rows; ++i) {
            double y = R_(i, j) + ubar[i];
            if (y > mx) mx = y;
        }
        if (mx == -INFINITY) {
            vbar[j] = INFINITY;
            bad += 1;
            continue;
        }
        double s = 0.0;
        for (int i = 0; i < rows; ++i) {
            double y = R_(i, j) + ubar[i];
            if (y != -INFINITY) s += exp(p * (y - mx));
        }
        vbar[j] = -mx - log(s) / p;
    }
    return bad;
}

/* Row sums r_i and column sums c_j of X = diag(u) A^(p) diag(v). */
void or_sums(int n, double p, const double *B, const double *ubar, const double *vbar,
             double *r, double *c)
{
#pragma omp parallel for schedule(static) if (n >= 128)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
            double b = B_(i, j);
            if (b != -INFINITY) s += exp(p * (b + ubar[i] + vbar[j]));
        }
        r[i] = s;
    }
#pragma omp parallel for schedule(static) if (n >= 128)
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) {
            double b = B_(i, j);
            if (b != -INFINITY) s += exp(p * (b + ubar[i] + vbar[j]));
        }
        c[j] = s;
    }
}

/* Distance of the column-stochastic iterate to bistochasticity: max_i |r_i - 1|
 * (Section 4.2, definition of an epsilon-bistochastic matrix). */
double or_row_residual(int n, double p, const double *B, const double *ubar, const double *vbar)
{
    double res = 0.0;
#pragma omp parallel for reduction(max : res) schedule(static) if (n >= 128)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
            double b = B_(i, j);
            if (b != -INFINITY) s += exp(p * (b + ubar[i] + vbar[j]));
        }
        double d = fabs(s - 1.0);
        if (!(d <= res)) res = d; /* NaN propagates as a failure */
    }
    return res;
}

/* Sinkhorn iteration on A^(p) (Section 3.1): starting from the given vbar
 * (vbar = 0 is v_0 = 1, eq. dad1), repeat a row step then a column step; the
 * iterate after m full iterations is W_m = diag(u_m) A^(p) diag(v_m), which is
 * column-stochastic. Stop as soon as max_i |r_i(W_m) - 1| < eps (strict), or
 * after max_iters iterations. ubar, vbar are in/out. Returns 0, or the number
 * of empty rows/columns met (no support). */
int or_sinkhorn(int n, double p, const double *B, double *ubar, double *vbar, double eps,
                long max_iters, long *iters_out, double *res_out)
{
    long m = 0;
    double res = INFINITY;
    int bad = 0;
    while (m < max_iters) {
        bad = or_row_step(n, n, p, B, vbar, ubar);
        if (bad) break;
        bad = or_col_step(n, n, p, B, ubar, vbar);
        if (bad) break;
        m += 1;
        res = or_row_residual(n, p, B, ubar, vbar);
        if (res < eps) break;
    }
    *iters_out = m;
    *res_out = res;
    return bad;
}

/* Continuation in p: scale A^(p) for each p of the ladder in turn. The
 * scalings are carried from one p to the next in the paper's log coordinates
 * (ubar, vbar held fixed), which is a warm start for the next Sinkhorn run;
 * by the uniqueness of X(p) (Theorem prop-borweinlewisnussbaum) the limit of
 * each stage does not depend on it. */
int or_scale_ladder(int n, const double *B, const double *ladder, int n_p, double eps,
                    long max_iters, double *ubar, double *vbar, long *iters, double *res)
{
    for (int k = 0; k < n_p; ++k) {
        int bad = or_sinkhorn(n, ladder[k], B, ubar, vbar, eps, max_iters, &iters[k], &res[k]);
        if (bad) return bad;
    }
    return 0;
}

/* Reduced matrix B of eq. matrixred: keep (i, j) iff x_ij(p) >= t.
 * keep[i*n+j] = 1 for kept entries. Returns the number kept. */
long or_prune(int n, double p, const double *B, const double *ubar, const double *vbar,
              double t, uint8_t *keep)
{
    long nnz = 0;
#pragma omp parallel for reduction(+ : nnz) schedule(static) if (n >= 128)
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            double b = B_(i, j);
            uint8_t k = 0;
            if (b != -INFINITY) {
                double x = exp(p * (b + ubar[i] + vbar[j]));
                k = (x >= t) ? 1 : 0;
            }
            keep[(size_t)i * n + j] = k;
            nnz += k;
        }
    }
    return nnz;
}

/* Approximate optimality certificate (Proposition prop:aoc): with
 * X = D_r A^(p) D_c, log x_ij = p (b_ij + ubar_i + vbar_j), log d_r,i = p ubar_i,
 * log d_c,j = p vbar_j,
 *   log omega_opt(A) <= p^-1 ( sum_i max_j log x_ij - sum_i log d_r,i - sum_j log d_c,j ).
 * Returns the right-hand side. The bound holds for any positive d_r, d_c. */
double or_certificate(int n, double p, const double *B, const double *ubar, const double *vbar)
{
    double s_max = 0.0, s_r = 0.0, s_c = 0.0;
    for (int i = 0; i < n; ++i) {
        double mx = -INFINITY;
        for (int j = 0; j < n; ++j) {
            double lx = p * (B_(i, j) + ubar[i] + vbar[j]);
            if (lx > mx) mx = lx;
        }
        s_max += mx;
    }
    for (int i = 0; i < n; ++i) s_r += p * ubar[i];
    for (int j = 0; j < n; ++j) s_c += p * vbar[j];
    return (s_max - s_r - s_c) / p;
}

/* Prescaling step of Section 4.1.1 on a linear matrix A (zeros allowed):
 * if max/min > e: m = 1/log(max/min), c = exp(log(min)/log(max/min)),
 * A <- A^(m) / c; otherwise A <- A / min. min is over positive entries. */
void or_prescale(int n, const double *A, double *out)
{
    double mx = 0.0, mn = INFINITY;
    for (size_t k = 0; k < (size_t)n * n; ++k) {
        if (A[k] > 0.0) {
            if (A[k] > mx) mx = A[k];
            if (A[k] < mn) mn = A[k];
        }
    }
    if (mx / mn > exp(1.0)) {
        double m = 1.0 / log(mx / mn);
        double c = exp(log(mn) / log(mx / mn));
        for (size_t k = 0; k < (size_t)n * n; ++k)
            out[k] = A[k] > 0.0 ? pow(A[k], m) / c : 0.0;
    } else {
        for (size_t k = 0; k < (size_t)n * n; ++k) out[k] = A[k] / mn;
    }
}

/* Exact optimal assignment, dense O(n^3) (the Kuhn/Edmonds class of solvers
 * cited in Section 1): Hungarian method with row/column potentials and
 * shortest augmenting paths, maximising sum_i w[i, perm(i)] over the allowed
 * entries. Returns 0 and fills perm/weight, or 1 if no perfect matching uses
 * only allowed entries. */
int or_hungarian(int n, const int64_t *w, const uint8_t *allowed, int32_t *perm, int64_t *weight)
{
    const int64_t INF = INT64_MAX / 4;
    /* 1-based arrays; column 0 is the virtual start of each search */
    int64_t *u = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *v = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *minv = malloc(((size_t)n + 1) * sizeof(int64_t));
    int *match = calloc((size_t)n + 1, sizeof(int)); /* match[j] = row of column j */
    int *way = calloc((size_t)n + 1, sizeof(int));
    char *used = malloc((size_t)n + 1);
    int status = 0;
    for (int i = 1; i <= n && status == 0; ++i) {
        match[0] = i;
        int j0 = 0;
        for (int j = 0; j <= n; ++j) {
            minv[j] = INF;
            used[j] = 0;
        }
        do {
            used[j0] = 1;
            int i0 = match[j0];
            int64_t delta = INF;
            int j1 = -1;
            for (int j = 1; j <= n; ++j) {
                if (used[j]) continue;
                size_t k = (size_t)(i0 - 1) * n + (size_t)(j - 1);
                if (allowed[k]) {
                    int64_t cur = -w[k] - u[i0] - v[j]; /* reduced cost of -w */
                    if (cur < minv[j]) {
                        minv[j] = cur;
                        way[j] = j0;
                    }
                }
                if (minv[j] < delta) {
                    delta = minv[j];
                    j1 = j;
                }
            }
            if (j1 < 0 || delta >= INF) {
                status = 1; /* no augmenting path: B has no perfect matching */
                break;
            }
            for (int j = 0; j <= n; ++j) {
                if (used[j]) {
                    u[match[j]] += delta;
                    v[j] -= delta;
                } else if (minv[j] < INF) {
                    minv[j] -= delta;
                }
            }
            j0 = j1;
        } while (match[j0] != 0);
        if (status) break;
        do {
            int j1 = way[j0];
            match[j0] = match[j1];
            j0 = j1;
        } while (j0);
    }
    if (status == 0) {
        int64_t total = 0;
        for (int j = 1; j <= n; ++j) {
            perm[match[j] - 1] = j - 1;
            total += w[(size_t)(match[j] - 1) * n + (size_t)(j - 1)];
        }
        *weight = total;
    }
    free(u);
    free(v);
    free(minv);
    free(match);
    free(way);
    free(used);
    return status;
}

/* The same dense O(n^3) Hungarian method for real weights (log-weights of a
 * nonnegative matrix), maximising sum_i w[i, perm(i)] over the allowed
 * entries in FP64. Returns 0 and fills perm/weight, or 1 if no perfect
 * matching uses only allowed entries. */
int or_hungarian_real(int n, const double *w, const uint8_t *allowed, int32_t *perm,
                      double *weight)
{
    double *u = calloc((size_t)n + 1, sizeof(double));
    double *v = calloc((size_t)n + 1, sizeof(double));
    double *minv = malloc(((size_t)n + 1) * sizeof(double));
    int *match = calloc((size_t)n + 1, sizeof(int));
    int *way = calloc((size_t)n + 1, sizeof(int));
    char *used = malloc((size_t)n + 1);
    int status = 0;
    for (int i = 1; i <= n && status == 0; ++i) {
        match[0] = i;
        int j0 = 0;
        for (int j = 0; j <= n; ++j) {
            minv[j] = INFINITY;
            used[j] = 0;
        }
        do {
            used[j0] = 1;
            int i0 = match[j0];
            double delta = INFINITY;
            int j1 = -1;
            for (int j = 1; j <= n; ++j) {
                if (used[j]) continue;
                size_t k = (size_t)(i0 - 1) * n + (size_t)(j - 1);
                if (allowed[k]) {
                    double cur = -w[k] - u[i0] - v[j];
                    if (cur < minv[j]) {
                        minv[j] = cur;
                        way[j] = j0;
                    }
                }
                if (minv[j] < delta) {
                    delta = minv[j];
                    j1 = j;
                }
            }
            if (j1 < 0 || delta == INFINITY) {
                status = 1;
                break;
            }
            for (int j = 0; j <= n; ++j) {
                if (used[j]) {
                    u[match[j]] += delta;
                    v[j] -= delta;
                } else if (minv[j] < INFINITY) {
                    minv[j] -= delta;
                }
            }
            j0 = j1;
        } while (match[j0] != 0);
        if (status) break;
        do {
            int j1 = way[j0];
            match[j0] = match[j1];
            j0 = j1;
        } while (j0);
    }
    if (status == 0) {
        double total = 0.0;
        for (int j = 1; j <= n; ++j) {
            perm[match[j] - 1] = j - 1;
            total += w[(size_t)(match[j] - 1) * n + (size_t)(j - 1)];
        }
        *weight = total;
    }
    free(u);
    free(v);
    free(minv);
    free(match);
    free(way);
    free(used);
    return status;
}
