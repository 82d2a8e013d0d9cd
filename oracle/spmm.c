/*
 * FP64 CPU oracle for the symmetric sparse-matrix x block-of-vectors product.
 *
 * TEST INFRASTRUCTURE ONLY: this code exists to check the HIP path and to
 * time a plain CPU baseline.  The product library never links or calls it.
 *
 * H is given by its upper triangle U (diagonal included) in CSR; the product
 * is the plain definition  Y = (U + U^T - diag(U)) X  in double precision,
 * with X and Y row-major n x k ("multiple vectors stored in row major order",
 * paper Section 3.3).  As in the paper's CPU code (Section 3.2, 3.3), the
 * product with the stored part and the product with its transpose are two
 * separate loops, each written as a race-free "pull" over output rows:
 *   pass 1 (rows):       Y_i  = sum_{j >= i} u_ij X_j
 *   pass 2 (transposed): Y_j += sum_{i <  j} u_ij X_i     (over a CSC copy of U)
 * Each entry contributes u_ij * X_j(:) to row i, the paper's update
 * U_i(r,:) += v * W_j(c,:) (Algorithm 2).  Rows are parallelised with OpenMP.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

typedef struct {
    int64_t n, nnz;
    int64_t *rp; int32_t *ci; double *v;       /* U, CSR, FP64 copy */
    int64_t *cp; int32_t *ri; double *cv;      /* strict upper part of U, CSC (= CSR of the strict lower part) */
} oracle_mat;

oracle_mat *oracle_mat_create(int64_t n, const int64_t *rp, const int32_t *col, const void *val, int val_is_f32) {
    oracle_mat *m = (oracle_mat *)calloc(1, sizeof(oracle_mat));
    if (!m) return NULL;
    m->n = n; m->nnz = rp[n];
    m->rp = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    m->ci = (int32_t *)malloc((size_t)(m->nnz ? m->nnz : 1) * sizeof(int32_t));
    m->v = (double *)malloc((size_t)(m->nnz ? m->nnz : 1) * sizeof(double));
    memcpy(m->rp, rp, ((size_t)n + 1) * sizeof(int64_t));
    memcpy(m->ci, col, (size_t)m->nnz * sizeof(int32_t));
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m->nnz; ++e)
        m->v[e] = val_is_f32 ? (double)((const float *)val)[e] : ((const double *)val)[e];
    /* CSC of the strict upper triangle */
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (col[e] != i) cnt[col[e] + 1]++;
    for (int64_t j = 0; j < n; ++j) cnt[j + 1] += cnt[j];
    m->cp = cnt;
    int64_t nt = cnt[n];
    m->ri = (int32_t *)malloc((size_t)(nt ? nt : 1) * sizeof(int32_t));
    m->cv = (double *)malloc((size_t)(nt ? nt : 1) * sizeof(double));
    int64_t *cur = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    memcpy(cur, cnt, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)               /* rows ascending -> each column's rows ascending */
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (col[e] != i) { int64_t p = cur[col[e]]++; m->ri[p] = (int32_t)i; m->cv[p] = m->v[e]; }
    free(cur);
    return m;
}

void oracle_mat_free(oracle_mat *m) {
    if (!m) return;
    free(m->rp); free(m->ci); free(m->v); free(m->cp); free(m->ri); free(m->cv); free(m);
}

/* Y = H X (use_abs = 0) or Y = |H| |X| (use_abs = 1, the scale that bounds rounding error) */
static void spmm_impl(const oracle_mat *m, int64_t k, const double *X, double *Y, int use_abs) {
    const int64_t n = m->n;
    /* pass 1: the stored part, row by row */
    #pragma omp parallel for schedule(dynamic, 512) if (m->nnz * k > 4000000)
    for (int64_t i = 0; i < n; ++i) {
        double *y = Y + i * k;
        for (int64_t q = 0; q < k; ++q) y[q] = 0.0;
        for (int64_t e = m->rp[i]; e < m->rp[i + 1]; ++e) {
            double a = use_abs ? fabs(m->v[e]) : m->v[e];
            const double *x = X + (int64_t)m->ci[e] * k;
            for (int64_t q = 0; q < k; ++q) y[q] += a * (use_abs ? fabs(x[q]) : x[q]);
        }
    }
    /* pass 2: the transposed part, pulled through the CSC copy */
    #pragma omp parallel for schedule(dynamic, 512) if (m->nnz * k > 4000000)
    for (int64_t j = 0; j < n; ++j) {
        double *y = Y + j * k;
        for (int64_t e = m->cp[j]; e < m->cp[j + 1]; ++e) {
            double a = use_abs ? fabs(m->cv[e]) : m->cv[e];
            const double *x = X + (int64_t)m->ri[e] * k;
            for (int64_t q = 0; q < k; ++q) y[q] += a * (use_abs ? fabs(x[q]) : x[q]);
        }
    }
}

void oracle_spmm(const oracle_mat *m, int64_t k, const double *X, double *Y) { spmm_impl(m, k, X, Y, 0); }
void oracle_spmm_abs(const oracle_mat *m, int64_t k, const double *X, double *Y) { spmm_impl(m, k, X, Y, 1); }

/* Selected rows of H X (and |H||X|): Yr[t,:] = row rows[t] of the product. */
void oracle_spmm_rows(const oracle_mat *m, int64_t k, const double *X, int64_t nrows, const int64_t *rows,
                      double *Yr, double *Yabs) {
    #pragma omp parallel for schedule(dynamic, 16) if (nrows * 64 > 100000)
    for (int64_t t = 0; t < nrows; ++t) {
        int64_t i = rows[t];
        double *y = Yr + t * k, *ya = Yabs ? Yabs + t * k : NULL;
        for (int64_t q = 0; q < k; ++q) { y[q] = 0.0; if (ya) ya[q] = 0.0; }
        for (int64_t e = m->rp[i]; e < m->rp[i + 1]; ++e) {
            const double *x = X + (int64_t)m->ci[e] * k;
            for (int64_t q = 0; q < k; ++q) { y[q] += m->v[e] * x[q]; if (ya) ya[q] += fabs(m->v[e]) * fabs(x[q]); }
        }
        for (int64_t e = m->cp[i]; e < m->cp[i + 1]; ++e) {
            const double *x = X + (int64_t)m->ri[e] * k;
            for (int64_t q = 0; q < k; ++q) { y[q] += m->cv[e] * x[q]; if (ya) ya[q] += fabs(m->cv[e]) * fabs(x[q]); }
        }
    }
}

/* Gershgorin bound on ||H||_2: max_i sum_j |H_ij| over full symmetric rows. */
double oracle_gershgorin(const oracle_mat *m) {
    double best = 0.0;
    #pragma omp parallel for schedule(dynamic, 1024) reduction(max : best)
    for (int64_t i = 0; i < m->n; ++i) {
        double s = 0.0;
        for (int64_t e = m->rp[i]; e < m->rp[i + 1]; ++e) s += fabs(m->v[e]);
        for (int64_t e = m->cp[i]; e < m->cp[i + 1]; ++e) s += fabs(m->cv[e]);
        if (s > best) best = s;
    }
    return best;
}

/* Full-row off-diagonal 1-norms sum_{j != i} |H_ij|. */
void oracle_row_offdiag_abs(const oracle_mat *m, double *out) {
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < m->n; ++i) {
        double s = 0.0;
        for (int64_t e = m->rp[i]; e < m->rp[i + 1]; ++e) if (m->ci[e] != i) s += fabs(m->v[e]);
        for (int64_t e = m->cp[i]; e < m->cp[i + 1]; ++e) s += fabs(m->cv[e]);
        out[i] = s;
    }
}

/* Full-row off-diagonal nonzero counts. */
void oracle_row_offdiag_count(const oracle_mat *m, int64_t *out) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->n; ++i) {
        int64_t c = 0;
        for (int64_t e = m->rp[i]; e < m->rp[i + 1]; ++e) if (m->ci[e] != i) ++c;
        out[i] = c + (m->cp[i + 1] - m->cp[i]);
    }
}

/* Thread count of the OpenMP loops above (timing of the CPU baseline only). */
void oracle_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
int oracle_get_threads(void) { return omp_get_max_threads(); }
