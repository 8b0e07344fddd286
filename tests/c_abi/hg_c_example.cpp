/*
 * The C boundary used from a host program with no Python: one field set up, gridded and
 * checked, as a caller linking libhegrid.so would.  Built by the package's
 * build step; run by tests/test_gpu_c_abi.py on a GPU.
 *
 * 3000 samples over a 0.2 x 0.5 deg box east of (30, 20) deg, a 24 x 24 map at
 * 1 arcmin, Gaussian FWHM 3 arcmin with 3 sigma support, 4 FP32 channels:
 * channel c holds the constant c + 1.5, so every cell with a neighbour must
 * come out as c + 1.5 (a weighted mean of equal values, to FP32 rounding of
 * the sums) and every cell without one as NaN.  Also checks an argument error
 * and hg_last_error, and prints "c abi ok" on success (exit status 0).
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "hegrid.h"

#define CHECK_HIP(x)                                                  \
    do {                                                              \
        hipError_t e_ = (x);                                          \
        if (e_ != hipSuccess) {                                       \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));   \
            return 2;                                                 \
        }                                                             \
    } while (0)

int main(void) {
    const int64_t n = 3000;
    const int32_t nx = 24, ny = 24, C = 4;
    double* ra = (double*)malloc(sizeof(double) * n);
    double* dec = (double*)malloc(sizeof(double) * n);
    float* vals = (float*)malloc(sizeof(float) * n * C);
    uint64_t s = 2207045840ull;
    for (int64_t i = 0; i < n; i++) {  /* a 64-bit LCG (Knuth's MMIX constants) */
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        double u = (double)(s >> 11) / 9007199254740992.0;
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        double v = (double)(s >> 11) / 9007199254740992.0;
        ra[i] = 30.0 + u * 0.2;  /* the map's eastern half only: its west stays empty */
        dec[i] = 20.0 + (v - 0.5) * 0.5;
        for (int c = 0; c < C; c++) vals[i * C + c] = (float)c + 1.5f;
    }
    double *d_ra, *d_dec;
    float *d_vals, *d_out;
    CHECK_HIP(hipMalloc((void**)&d_ra, sizeof(double) * n));
    CHECK_HIP(hipMalloc((void**)&d_dec, sizeof(double) * n));
    CHECK_HIP(hipMalloc((void**)&d_vals, sizeof(float) * n * C));
    CHECK_HIP(hipMalloc((void**)&d_out, sizeof(float) * C * nx * ny));
    CHECK_HIP(hipMemcpy(d_ra, ra, sizeof(double) * n, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_dec, dec, sizeof(double) * n, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_vals, vals, sizeof(float) * n * C, hipMemcpyHostToDevice));

    const double fwhm = 3.0 / 60.0;
    hg_kernel k = {fwhm, 3.0 * fwhm / sqrt(8.0 * log(2.0)), HG_KERNEL_GAUSS, 0, 0.0, 0.0};
    hg_map m = {30.0, 20.0, 1.0 / 60.0, 1.0 / 60.0, nx, ny};
    hg_plan* plan = NULL;
    int rc = hg_grid_setup(d_ra, d_dec, n, &k, &m, NULL, NULL, &plan);
    if (rc != HG_OK) {
        fprintf(stderr, "hg_grid_setup: %d %s\n", rc, hg_last_error());
        return 1;
    }
    rc = hg_grid_channels(plan, d_vals, C, C, HG_F32, d_out, NULL);
    if (rc != HG_OK) {
        fprintf(stderr, "hg_grid_channels: %d %s\n", rc, hg_last_error());
        return 1;
    }
    CHECK_HIP(hipDeviceSynchronize());
    float* out = (float*)malloc(sizeof(float) * C * nx * ny);
    int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * nx * ny);
    CHECK_HIP(hipMemcpy(out, d_out, sizeof(float) * C * nx * ny, hipMemcpyDeviceToHost));
    if (hg_plan_counts(plan, cnt) != HG_OK) {
        fprintf(stderr, "hg_plan_counts: %s\n", hg_last_error());
        return 1;
    }
    int filled = 0, empty = 0;
    for (int p = 0; p < nx * ny; p++) {
        if (cnt[p] > 0) filled++; else empty++;
        for (int c = 0; c < C; c++) {
            float v = out[c * nx * ny + p];
            float want = (float)c + 1.5f;
            if (cnt[p] > 0 ? !(fabsf(v - want) <= 1e-5f * want) : !isnan(v)) {
                fprintf(stderr, "cell %d channel %d: %g (count %d)\n", p, c, v, cnt[p]);
                return 1;
            }
        }
    }
    if (filled == 0 || empty == 0) {
        fprintf(stderr, "expected both filled and empty cells: %d %d\n", filled, empty);
        return 1;
    }
    /* an argument error leaves a message and no work */
    rc = hg_grid_channels(plan, d_vals, C - 1, C, HG_F32, d_out, NULL);
    if (rc != HG_ERR_ARG || hg_last_error()[0] == 0) {
        fprintf(stderr, "ld < nchan was not rejected (%d)\n", rc);
        return 1;
    }
    if (hg_grid_finish(plan) != HG_OK) return 1;
    printf("c abi ok: %d cells with neighbours, %d without\n", filled, empty);
    return 0;
}
