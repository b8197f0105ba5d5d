/* The C ABI used from plain C, without Python: reads a squared-Euclidean problem from a
 * binary file, runs lamp_solve for a fixed number of iterations, takes lamp_certificate
 * of the result, and writes nu, theta and the certificate's transport cost.
 *
 * usage: solve_example IN OUT T ETA
 *   IN:  int64 n, int64 m, int32 d, then x (n d float32), y (m d float32), r (n float64),
 *        c (m float64)
 *   OUT: nu (m float64), theta (m float64), cost (float64), t (int64)
 * Exit status 0 on success, 2 on a library error (message on stderr), 3 on an I/O or
 * HIP runtime error. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "lamp.h"

#define HIPOK(call)                                                               \
    do {                                                                          \
        if ((call) != hipSuccess) {                                               \
            fprintf(stderr, "HIP call failed: %s (line %d)\n", #call, __LINE__); \
            return 3;                                                             \
        }                                                                         \
    } while (0)

static int read_all(FILE* f, void* p, size_t bytes) { return fread(p, 1, bytes, f) == bytes; }

int main(int argc, char** argv) {
    if (argc != 5) {
        fprintf(stderr, "usage: %s IN OUT T ETA\n", argv[0]);
        return 3;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 3;
    int64_t n, m;
    int32_t d;
    if (!read_all(f, &n, 8) || !read_all(f, &m, 8) || !read_all(f, &d, 4)) return 3;
    const size_t bx = sizeof(float) * (size_t)n * (size_t)d, by = sizeof(float) * (size_t)m * (size_t)d;
    float* x = malloc(bx);
    float* y = malloc(by);
    double* r = malloc(sizeof(double) * (size_t)n);
    double* c = malloc(sizeof(double) * (size_t)m);
    double* out = malloc(sizeof(double) * 2 * (size_t)m);
    if (!x || !y || !r || !c || !out) return 3;
    if (!read_all(f, x, bx) || !read_all(f, y, by) || !read_all(f, r, sizeof(double) * (size_t)n) ||
        !read_all(f, c, sizeof(double) * (size_t)m))
        return 3;
    fclose(f);

    float *dx, *dy;
    double *dr, *dc, *dnu, *dth;
    void* ws;
    HIPOK(hipMalloc((void**)&dx, bx));
    HIPOK(hipMalloc((void**)&dy, by));
    HIPOK(hipMalloc((void**)&dr, sizeof(double) * (size_t)n));
    HIPOK(hipMalloc((void**)&dc, sizeof(double) * (size_t)m));
    HIPOK(hipMalloc((void**)&dnu, sizeof(double) * (size_t)m));
    HIPOK(hipMalloc((void**)&dth, sizeof(double) * (size_t)m));
    HIPOK(hipMemcpy(dx, x, bx, hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(dy, y, by, hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(dr, r, sizeof(double) * (size_t)n, hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(dc, c, sizeof(double) * (size_t)m, hipMemcpyHostToDevice));
    HIPOK(hipMemset(dnu, 0, sizeof(double) * (size_t)m));   /* t = 0, nu = theta = 0: a fresh start */
    HIPOK(hipMemset(dth, 0, sizeof(double) * (size_t)m));

    lamp_problem prob = {n, m, d, LAMP_SQEUCLID, dx, dy, dr, dc, 0.0, 0.0, NULL, LAMP_COST_F32, 0};
    lamp_params params = {atof(argv[4]), 0.0, atoll(argv[3]), 0.0, 0.0, 0.0, 0.0, LAMP_FP32, 16, 0, 0};
    lamp_state state = {dnu, dth, 0, 0.0, 0.0};
    const size_t ws_bytes = lamp_workspace_bytes(&prob, &params);
    if (ws_bytes == 0) return 2;
    HIPOK(hipMalloc(&ws, ws_bytes));   /* hipMalloc returns at least 256-byte aligned memory */

    lamp_report rep;
    lamp_status s = lamp_solve(&prob, &params, &state, ws, ws_bytes, NULL, &rep);
    if (s != LAMP_OK) {
        fprintf(stderr, "lamp_solve: %d %s\n", (int)s, lamp_last_error());
        return 2;
    }
    lamp_cert cert;
    s = lamp_certificate(&prob, &params, &state, ws, ws_bytes, NULL, &cert);
    if (s != LAMP_OK) {
        fprintf(stderr, "lamp_certificate: %d %s\n", (int)s, lamp_last_error());
        return 2;
    }
    HIPOK(hipMemcpy(out, dnu, sizeof(double) * (size_t)m, hipMemcpyDeviceToHost));
    HIPOK(hipMemcpy(out + m, dth, sizeof(double) * (size_t)m, hipMemcpyDeviceToHost));
    f = fopen(argv[2], "wb");
    if (!f) return 3;
    fwrite(out, sizeof(double), 2 * (size_t)m, f);
    fwrite(&cert.cost, sizeof(double), 1, f);
    fwrite(&state.t, sizeof(int64_t), 1, f);
    fclose(f);
    printf("solve_example: t = %lld, final residual %.3e, cost %.12e\n", (long long)state.t, rep.final_res,
           cert.cost);
    HIPOK(hipFree(ws));
    HIPOK(hipFree(dx));
    HIPOK(hipFree(dy));
    HIPOK(hipFree(dr));
    HIPOK(hipFree(dc));
    HIPOK(hipFree(dnu));
    HIPOK(hipFree(dth));
    free(x);
    free(y);
    free(r);
    free(c);
    free(out);
    return 0;
}
