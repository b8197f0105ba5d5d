/* Full-size marginal passes of one LAMP iteration in FP64, plain C with OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY (oracle): the row log-normalisers and sampled column
 * marginals of p^{1/lam}(v) (Section 4.1, first and second display) at sizes where
 * NumPy is too slow, for the parity checks of large workloads.
 *
 * Cost C_ij = s * c_ij with, per `form`:
 *   form 0: c_ij = ||x_i - y_j||^2, difference form of the FP32 points, every
 *           coordinate promoted exactly to FP64 before the subtraction;
 *   form 1: c_ij = nx_i + ny_j - 2 sum_k xr_ik yr_jk from FP64 arrays (the cost a
 *           caller defines by rounded inner products and separate squared norms).
 * For coupling q (q < nc) with dual v_q (m values) and inverse temperature lam_q:
 *   a^q_ij = -lam_q (C_ij + K v_q,j),
 *   logZ^q_i = max_j a^q_ij + log sum_j exp(a^q_ij - max_j a^q_ij)      (oracle_log_normalisers)
 *   col^q_j = sum_i r_i exp(a^q_ij - logZ^q_i)   for the listed columns  (oracle_sampled_columns)
 *   E^q_i = sum_j exp(a^q_ij - logZ^q_i) C_ij    for every row          (oracle_row_costs),
 *           so that <C, diag(r) p^{1/lam_q}(v_q)> = sum_i r_i E^q_i
 * Each row (each listed column) is evaluated by one thread, so results do not
 * depend on the number of threads.  Built with -ffast-math so that the sum of
 * exponentials vectorises (partial sums in SIMD lanes): a change of rounding order
 * only, at FP64; every input is finite.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int32_t form, d;
    int64_t n, m;
    const float *x, *y;        /* form 0: n x d, m x d */
    const double *xr, *yr;     /* form 1: n x d, m x d */
    const double *nx, *ny;     /* form 1: n, m */
    double s, K;
} cost_def;

__attribute__((target_clones("avx2", "default")))
static double cost_entry(const cost_def *c, int64_t i, int64_t j)
{
    double acc = 0.0;
    if (c->form == 0) {
        const float *xi = c->x + i * c->d, *yj = c->y + j * c->d;
        for (int32_t k = 0; k < c->d; ++k) {
            double diff = (double)xi[k] - (double)yj[k];
            acc += diff * diff;
        }
    } else {
        const double *xi = c->xr + i * c->d, *yj = c->yr + j * c->d;
        double dot = 0.0;
        for (int32_t k = 0; k < c->d; ++k) dot += xi[k] * yj[k];
        acc = c->nx[i] + c->ny[j] - 2.0 * dot;
    }
    return c->s * acc;
}

/* row[j] = C_ij for j < m. */
__attribute__((target_clones("avx2", "default")))
static void cost_row(const cost_def *c, int64_t i, double *row)
{
    if (c->form == 0) {
        const float *xi = c->x + i * c->d;
        for (int64_t j = 0; j < c->m; ++j) {
            const float *yj = c->y + j * c->d;
            double acc = 0.0;
            for (int32_t k = 0; k < c->d; ++k) {
                double diff = (double)xi[k] - (double)yj[k];
                acc += diff * diff;
            }
            row[j] = c->s * acc;
        }
    } else {
        const double *xi = c->xr + i * c->d;
        for (int64_t j = 0; j < c->m; ++j) {
            const double *yj = c->yr + j * c->d;
            double dot = 0.0;
            for (int32_t k = 0; k < c->d; ++k) dot += xi[k] * yj[k];
            row[j] = c->s * (c->nx[i] + c->ny[j] - 2.0 * dot);
        }
    }
}

/* sum_j exp(a_j - mx); built for AVX2 where the CPU has it (a SIMD exp from the C library,
 * FP64, within a few ulp) and plain otherwise. */
__attribute__((target_clones("avx2", "default")))
static double sum_exp_shifted(const double *a, int64_t m, double mx)
{
    double sum = 0.0;
#pragma omp simd reduction(+ : sum)
    for (int64_t j = 0; j < m; ++j) sum += exp(a[j] - mx);
    return sum;
}

void oracle_log_normalisers(const cost_def *c, int32_t nc, const double *v, const double *lam,
                            double *logZ)
{
#pragma omp parallel
    {
        double *row = (double *)malloc(sizeof(double) * (size_t)c->m);
        double *arg = (double *)malloc(sizeof(double) * (size_t)c->m);
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < c->n; ++i) {
            cost_row(c, i, row);
            for (int32_t q = 0; q < nc; ++q) {
                const double *vq = v + (int64_t)q * c->m;
                for (int64_t j = 0; j < c->m; ++j) arg[j] = -lam[q] * (row[j] + c->K * vq[j]);
                double mx = arg[0];
                for (int64_t j = 1; j < c->m; ++j)
                    if (arg[j] > mx) mx = arg[j];
                logZ[(int64_t)q * c->n + i] = mx + log(sum_exp_shifted(arg, c->m, mx));
            }
        }
        free(arg);
        free(row);
    }
}

/* acc[k] += r_i exp(-lam (C_{i,cols[k]} + K v_{cols[k]}) - logZ_i) for k < cnt, one row i. */
__attribute__((target_clones("avx2", "default")))
static void column_terms(const cost_def *c, int64_t i, const int64_t *cols, int64_t cnt, const double *v,
                         double lam, double Li, double ri, double *acc)
{
#pragma omp simd
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t j = cols[k];
        acc[k] += ri * exp(-lam * (cost_entry(c, i, j) + c->K * v[j]) - Li);
    }
}

void oracle_sampled_columns(const cost_def *c, int32_t nc, const double *v, const double *lam,
                            const double *logZ, const double *r, const int64_t *cols, int64_t ncols,
                            double *out)
{
    const int64_t CH = 64;    /* listed columns per task; each task walks every row in order */
    const int64_t ntask = (ncols + CH - 1) / CH;
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int32_t q = 0; q < nc; ++q) {
        for (int64_t tk = 0; tk < ntask; ++tk) {
            const int64_t k0 = tk * CH;
            const int64_t cnt = ncols - k0 < CH ? ncols - k0 : CH;
            double acc[64];
            for (int64_t k = 0; k < cnt; ++k) acc[k] = 0.0;
            const double *vq = v + (int64_t)q * c->m;
            const double *Lq = logZ + (int64_t)q * c->n;
            for (int64_t i = 0; i < c->n; ++i) column_terms(c, i, cols + k0, cnt, vq, lam[q], Lq[i], r[i], acc);
            for (int64_t k = 0; k < cnt; ++k) out[(int64_t)q * ncols + k0 + k] = acc[k];
        }
    }
}

/* sum_j exp(a_j - L) w_j */
__attribute__((target_clones("avx2", "default")))
static double sum_exp_weighted(const double *a, const double *w, int64_t m, double L)
{
    double sum = 0.0;
#pragma omp simd reduction(+ : sum)
    for (int64_t j = 0; j < m; ++j) sum += exp(a[j] - L) * w[j];
    return sum;
}

void oracle_row_costs(const cost_def *c, int32_t nc, const double *v, const double *lam, const double *logZ,
                      double *out)
{
#pragma omp parallel
    {
        double *row = (double *)malloc(sizeof(double) * (size_t)c->m);
        double *arg = (double *)malloc(sizeof(double) * (size_t)c->m);
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < c->n; ++i) {
            cost_row(c, i, row);
            for (int32_t q = 0; q < nc; ++q) {
                const double *vq = v + (int64_t)q * c->m;
                for (int64_t j = 0; j < c->m; ++j) arg[j] = -lam[q] * (row[j] + c->K * vq[j]);
                out[(int64_t)q * c->n + i] = sum_exp_weighted(arg, row, c->m, logZ[(int64_t)q * c->n + i]);
            }
        }
        free(arg);
        free(row);
    }
}

#include <omp.h>

/* Threads an OpenMP parallel region of this library uses. */
int oracle_num_threads(void) { return omp_get_max_threads(); }
