/* max_ij ||x_i - y_j||^2 in FP64, difference form, plain C with OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY (oracle): used to fix the cost normalisation
 * s = 1 / max_ij ||x_i - y_j||^2 (so that ||C||_inf = 1) of large synthetic
 * workloads.  x is n x d and y is m x d, row-major FP32; every coordinate is
 * promoted exactly to FP64 before the subtraction.
 */
#include <stdint.h>

double oracle_max_sqdist(const float *x, const float *y, int64_t n, int64_t m, int32_t d)
{
    double best = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : best)
    for (int64_t i = 0; i < n; ++i) {
        const float *xi = x + i * d;
        double row_best = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            const float *yj = y + j * d;
            double acc = 0.0;
            for (int32_t k = 0; k < d; ++k) {
                double diff = (double)xi[k] - (double)yj[k];
                acc += diff * diff;
            }
            if (acc > row_best) row_best = acc;
        }
        if (row_best > best) best = row_best;
    }
    return best;
}
