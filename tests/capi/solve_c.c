/* Drives the reconstruction through the C ABI alone (no Python): a noiseless
 * 4-phase 32x32 disk phantom is projected with tnlm_project, solved from the
 * FBP of all phases with tnlm_solve, and checked: status, iteration count,
 * history length, finite output, a data term below that of the start, and
 * the argument-error path of tnlm_recon_init. Prints one line; exit 0 = pass. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tnlm.h"

enum { N = 4, SIDE = 32, V = 24, B = 48, K = 10 };
static const double kPi = 3.14159265358979323846;

static int fail(const char *what) {
    printf("capi FAIL: %s (%s)\n", what, tnlm_last_error());
    return 1;
}

int main(void) {
    double ang[N * V];
    for (int i = 0; i < N; ++i)
        for (int v = 0; v < V; ++v) ang[i * V + v] = 2.0 * kPi * (v + (double)i / N) / V;
    tnlm_geometry g;
    g.n_phases = N;
    g.L = SIDE;
    g.pixel_mm = 500.0 / SIDE;
    g.n_views = V;
    g.n_bins = B;
    g.sad_mm = 541.0;
    g.sdd_mm = 949.075;
    g.dgamma_rad = 888.0 * 1.0239 / 949.075 / B;
    g.det_offset_bins = 0.25;
    g.view_angles_rad = ang;
    tnlm_params p;
    p.patch = 3;
    p.window = 7;
    p.h = 0.02f;
    p.mu_hat = 0.5f;
    p.beta = 1.0f;
    p.m1_cgls = 3;
    p.m2_jacobi = 1;
    p.max_outer = K;
    p.tol_rel_update = 0.0f;
    p.init = TNLM_INIT_FBP_ALL;
    p.ssd_mode = TNLM_SSD_FP32;

    /* argument errors come back as status codes, with a message */
    tnlm_ctx *bad = NULL;
    tnlm_params pb = p;
    pb.patch = 4;
    if (tnlm_recon_init(&bad, &g, &pb, NULL) != TNLM_E_INVALID_ARG || bad != NULL || !tnlm_last_error()[0])
        return fail("even patch size accepted");

    tnlm_ctx *ctx = NULL;
    if (tnlm_recon_init(&ctx, &g, &p, NULL) != TNLM_OK) return fail("init");

    const int L = SIDE;
    const size_t ni = (size_t)N * L * L, ns = (size_t)N * V * B;
    float *hf = (float *)malloc(ni * sizeof(float)), *hw = (float *)malloc(ns * sizeof(float));
    for (int i = 0; i < N; ++i)   /* disk of radius L/4, centre moving one pixel per phase */
        for (int r = 0; r < L; ++r)
            for (int c = 0; c < L; ++c) {
                const double x = c - L / 2 + 0.5 - 0.5 * i, y = r - L / 2 + 0.5;
                hf[(size_t)i * L * L + r * L + c] = (x * x + y * y < (L / 4.0) * (L / 4.0)) ? 0.02f : 0.0f;
            }
    for (size_t k = 0; k < ns; ++k) hw[k] = 1.0f;
    float *d_true, *d_y, *d_w, *d_f, *d_f0;
    if (hipMalloc((void **)&d_true, ni * 4) || hipMalloc((void **)&d_f, ni * 4) || hipMalloc((void **)&d_f0, ni * 4) ||
        hipMalloc((void **)&d_y, ns * 4) || hipMalloc((void **)&d_w, ns * 4))
        return fail("hipMalloc");
    if (hipMemcpy(d_true, hf, ni * 4, hipMemcpyHostToDevice) || hipMemcpy(d_w, hw, ns * 4, hipMemcpyHostToDevice))
        return fail("hipMemcpy");
    if (tnlm_project(ctx, d_true, d_y) != TNLM_OK) return fail("project");
    if (tnlm_fbp(ctx, d_y, d_f0, 1) != TNLM_OK) return fail("fbp");
    double cost0 = 0.0, cost1 = 0.0;
    if (tnlm_data_cost(ctx, d_y, d_w, d_f0, &cost0) != TNLM_OK) return fail("data cost of the start");

    int32_t iters = 0;
    float rel = 0.0f;
    if (tnlm_solve(ctx, d_y, d_w, d_f, &iters, &rel) != TNLM_OK) return fail("solve");
    float hist[K];
    int32_t nh = 0;
    if (tnlm_get_history(ctx, hist, K, &nh) != TNLM_OK) return fail("history");
    if (tnlm_data_cost(ctx, d_y, d_w, d_f, &cost1) != TNLM_OK) return fail("data cost of the result");
    float *out = (float *)malloc(ni * sizeof(float));
    if (hipMemcpy(out, d_f, ni * 4, hipMemcpyDeviceToHost)) return fail("copy back");
    double e2 = 0.0, t2 = 0.0;
    int finite = 1;
    for (size_t k = 0; k < ni; ++k) {
        finite &= isfinite(out[k]) != 0;
        e2 += (out[k] - hf[k]) * (double)(out[k] - hf[k]);
        t2 += hf[k] * (double)hf[k];
    }
    const double err = sqrt(e2 / t2);
    printf("capi: iterations %d, history %d, last rel update %.3e, data term %.4e -> %.4e, rel error to phantom %.3f\n",
           iters, nh, rel, cost0, cost1, err);
    tnlm_destroy(ctx);
    hipFree(d_true);
    hipFree(d_f);
    hipFree(d_f0);
    hipFree(d_y);
    hipFree(d_w);
    free(hf);
    free(hw);
    free(out);
    if (iters != K || nh != K || !finite) return fail("iterations, history or finiteness");
    if (!(cost1 < cost0)) return fail("data term did not decrease");
    if (!(err < 0.5)) return fail("result far from the phantom");
    printf("capi ok\n");
    return 0;
}
