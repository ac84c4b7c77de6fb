// Host side of the C ABI declared in include/tnlm.h: argument validation,
// geometry tables, scratch ownership, and the enqueue order of one outer
// iteration of the TNLM algorithm box (§2.2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace tnlm;

namespace {

thread_local std::string g_last_error;

tnlm_status fail(tnlm_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? TNLM_E_OOM : TNLM_E_HIP,                       \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                        \
    } while (0)

}  // namespace

struct tnlm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    tnlm_geometry geom{};
    std::vector<double> angles;
    tnlm_params prm{};
    DevGeom dg{};
    RegShape rs{};
    std::vector<void *> allocs;
    float4 *rt0 = nullptr, *rt1 = nullptr, *vt = nullptr;
    float *hfilt = nullptr, *cw = nullptr;
    CglsBufs cb{};
    float *Q = nullptr;         // filtered sinogram / Eq. 4 scratch [N][V][B]
    float *ua = nullptr, *ub = nullptr;   // Gauss-Jacobi ping-pong [N][L][L]
    double *relpart = nullptr;
    int nrelblk = 0;
    int *flags = nullptr;       // [0] zero, [1] done, [2] counter, [3] nonfinite
    float *hist = nullptr;      // [max_outer]
    size_t nimg = 0, nsino = 0;

    // kernel timing (HIP events around every launch on the context's stream)
    struct TimedRec {
        int kind;
        hipEvent_t a, b;
    };
    bool timing = false;
    std::vector<TimedRec> recs;
    std::vector<hipEvent_t> pool;
    TimedRec pending{};
    hipEvent_t take_event() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else {
            (void)hipEventCreate(&e);
        }
        return e;
    }
    void tbegin(int kind) {
        if (!timing) return;
        pending.kind = kind;
        pending.a = take_event();
        pending.b = take_event();
        (void)hipEventRecord(pending.a, stream);
    }
    void tend() {
        if (!timing) return;
        (void)hipEventRecord(pending.b, stream);
        recs.push_back(pending);
    }

    template <class T>
    hipError_t alloc(T **p, size_t count) {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) {
            allocs.push_back(q);
            *p = (T *)q;
        }
        return e;
    }
    ~tnlm_ctx() {
        for (auto &r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
        for (void *p : allocs) (void)hipFree(p);
    }
    int *zero() { return flags + 0; }
    int *done() { return flags + 1; }
    int *counter() { return flags + 2; }
    int *nonfinite() { return flags + 3; }
};

static tnlm_status validate(const tnlm_geometry *g, const tnlm_params *p) {
    if (!g || !p) return fail(TNLM_E_INVALID_ARG, "null geometry or params");
    if (g->n_phases < 1 || g->L < 1 || g->L > 4096 || g->n_views < 1 || g->n_bins < 1 || g->n_bins > 4096)
        return fail(TNLM_E_SHAPE, "need N >= 1, 1 <= L <= 4096, V >= 1, 1 <= B <= 4096");
    if (!(g->pixel_mm > 0) || !(g->sad_mm > 0) || !(g->dgamma_rad > 0) || !g->view_angles_rad)
        return fail(TNLM_E_INVALID_ARG, "need pixel_mm, sad_mm, dgamma_rad > 0 and view angles");
    if (!std::isfinite(g->det_offset_bins)) return fail(TNLM_E_INVALID_ARG, "det_offset_bins not finite");
    const double half_diag = 0.7071067811865476 * g->pixel_mm * g->L;
    if (!(g->sad_mm > half_diag)) return fail(TNLM_E_INVALID_ARG, "source circle must enclose the image square");
    for (long k = 0; k < (long)g->n_phases * g->n_views; ++k)
        if (!std::isfinite(g->view_angles_rad[k])) return fail(TNLM_E_NONFINITE, "non-finite view angle");
    if (!(p->patch & 1) || !(p->window & 1) || !reg_supported(p->patch, p->window))
        return fail(TNLM_E_INVALID_ARG, "patch must be odd in [3,9], window odd in [3,21]");
    if (p->window > g->L) return fail(TNLM_E_SHAPE, "window larger than the image");
    if (!(p->h > 0) || !std::isfinite(p->h)) return fail(TNLM_E_INVALID_ARG, "h must be > 0");
    if (!(p->mu_hat >= 0) || !std::isfinite(p->mu_hat)) return fail(TNLM_E_INVALID_ARG, "mu_hat must be >= 0");
    if (!(p->beta > 0) || !std::isfinite(p->beta)) return fail(TNLM_E_INVALID_ARG, "beta must be > 0");
    if (p->m1_cgls < 0 || p->m1_cgls > 64) return fail(TNLM_E_INVALID_ARG, "m1_cgls must be in [0, 64]");
    if (p->m2_jacobi < 1 || p->m2_jacobi > 1000) return fail(TNLM_E_INVALID_ARG, "m2_jacobi must be in [1, 1000]");
    if (p->max_outer < 1 || p->max_outer > 100000) return fail(TNLM_E_INVALID_ARG, "max_outer must be >= 1");
    if (!(p->tol_rel_update >= 0)) return fail(TNLM_E_INVALID_ARG, "tol_rel_update must be >= 0");
    if (p->init != TNLM_INIT_FBP_ALL && p->init != TNLM_INIT_USER) return fail(TNLM_E_INVALID_ARG, "bad init");
    if (p->ssd_mode != TNLM_SSD_FP32 && p->ssd_mode != TNLM_SSD_BF16_MFMA)
        return fail(TNLM_E_INVALID_ARG, "bad ssd_mode");
    return TNLM_OK;
}

// Per-ray plane tables in double precision, rounded once to float.
static void build_tables(const tnlm_geometry &g, std::vector<float4> &rt0, std::vector<float4> &rt1,
                         std::vector<float4> &vt, std::vector<float> &hf, std::vector<float> &cw) {
    const int N = g.n_phases, V = g.n_views, B = g.n_bins, L = g.L;
    const double D = g.pixel_mm, X0 = -0.5 * D * L;
    rt0.resize((size_t)N * V * B);
    rt1.resize((size_t)N * V * B);
    vt.resize((size_t)N * V);
    for (int i = 0; i < N; ++i)
        for (int v = 0; v < V; ++v) {
            const double th = g.view_angles_rad[(size_t)i * V + v];
            const double sx = g.sad_mm * std::cos(th), sy = g.sad_mm * std::sin(th);
            vt[(size_t)i * V + v] = make_float4((float)sx, (float)sy, (float)std::cos(th), (float)std::sin(th));
            for (int b = 0; b < B; ++b) {
                const double gam = ((double)b - 0.5 * (B - 1) + g.det_offset_bins) * g.dgamma_rad;
                const double ux = std::cos(th + M_PI + gam), uy = std::sin(th + M_PI + gam);
                const double ts = -(sx * ux + sy * uy);   // source -> point nearest the centre
                const double ox = sx + ts * ux, oy = sy + ts * uy;
                const double ix = std::fabs(ux) > 1e-9 ? 1.0 / ux : std::copysign(1e9, ux == 0 ? 1.0 : ux);
                const double iy = std::fabs(uy) > 1e-9 ? 1.0 / uy : std::copysign(1e9, uy == 0 ? 1.0 : uy);
                const size_t k = ((size_t)i * V + v) * B + b;
                rt0[k] = make_float4((float)(D * ix), (float)((X0 - ox) * ix), (float)(D * iy), (float)((X0 - oy) * iy));
                rt1[k] = make_float4((float)ox, (float)oy, (float)ux, (float)uy);
            }
        }
    hf.resize(2 * (size_t)B - 1);
    const double a = g.dgamma_rad;
    for (int m = -(B - 1); m <= B - 1; ++m) {
        double h;
        if (m == 0) h = 1.0 / (8.0 * a * a);
        else if (m % 2 == 0) h = 0.0;
        else {
            const double s = std::sin(m * a);
            h = -1.0 / (2.0 * M_PI * M_PI * s * s);
        }
        hf[m + B - 1] = (float)(a * h);
    }
    cw.resize(B);
    for (int b = 0; b < B; ++b)
        cw[b] = (float)(g.sad_mm * std::cos(((double)b - 0.5 * (B - 1) + g.det_offset_bins) * a));
}

extern "C" tnlm_status tnlm_recon_init(tnlm_ctx **out, const tnlm_geometry *geom, const tnlm_params *params,
                                       void *stream) {
    if (!out) return fail(TNLM_E_INVALID_ARG, "null output pointer");
    *out = nullptr;
    tnlm_status s = validate(geom, params);
    if (s != TNLM_OK) return s;
    if (params->ssd_mode == TNLM_SSD_BF16_MFMA)
        return fail(TNLM_E_INVALID_ARG, "ssd_mode BF16_MFMA is not available in this build");
    auto *c = new (std::nothrow) tnlm_ctx();
    if (!c) return fail(TNLM_E_OOM, "host allocation failed");
    std::unique_ptr<tnlm_ctx> guard(c);
    HIP_TRY(hipGetDevice(&c->device));
    c->stream = (hipStream_t)stream;
    c->geom = *geom;
    const int N = geom->n_phases, L = geom->L, V = geom->n_views, B = geom->n_bins;
    c->angles.assign(geom->view_angles_rad, geom->view_angles_rad + (size_t)N * V);
    c->geom.view_angles_rad = c->angles.data();
    c->prm = *params;
    c->nimg = (size_t)N * L * L;
    c->nsino = (size_t)N * V * B;

    std::vector<float4> rt0, rt1, vt;
    std::vector<float> hf, cw;
    build_tables(c->geom, rt0, rt1, vt, hf, cw);
    HIP_TRY(c->alloc(&c->rt0, rt0.size()));
    HIP_TRY(c->alloc(&c->rt1, rt1.size()));
    HIP_TRY(c->alloc(&c->vt, vt.size()));
    HIP_TRY(c->alloc(&c->hfilt, hf.size()));
    HIP_TRY(c->alloc(&c->cw, cw.size()));
    HIP_TRY(hipMemcpy(c->rt0, rt0.data(), rt0.size() * sizeof(float4), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->rt1, rt1.data(), rt1.size() * sizeof(float4), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->vt, vt.data(), vt.size() * sizeof(float4), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->hfilt, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->cw, cw.data(), cw.size() * sizeof(float), hipMemcpyHostToDevice));

    DevGeom &d = c->dg;
    d.N = N; d.L = L; d.V = V; d.B = B;
    d.D = (float)geom->pixel_mm;
    d.X0 = (float)(-0.5 * geom->pixel_mm * L);
    d.dgamma = (float)geom->dgamma_rad;
    d.ucenter = (float)(0.5 * (B - 1) - geom->det_offset_bins);
    d.rt0 = c->rt0; d.rt1 = c->rt1; d.vt = c->vt;
    c->rs = RegShape{N, L, params->patch, params->window, params->h, params->mu_hat};

    CglsBufs &b = c->cb;
    b.nbp = bp_blocks_per_phase(d);
    b.npp = proj_blocks_per_phase(d);
    HIP_TRY(c->alloc(&b.u, c->nimg));
    HIP_TRY(c->alloc(&b.s, c->nimg));
    HIP_TRY(c->alloc(&b.t, c->nimg));
    HIP_TRY(c->alloc(&b.r, c->nsino));
    HIP_TRY(c->alloc(&b.q, c->nsino));
    HIP_TRY(c->alloc(&b.rw, c->nsino));
    HIP_TRY(c->alloc(&b.sw, c->nsino));
    HIP_TRY(c->alloc(&b.gpart[0], (size_t)N * b.nbp));
    HIP_TRY(c->alloc(&b.gpart[1], (size_t)N * b.nbp));
    HIP_TRY(c->alloc(&b.qpart, (size_t)N * b.npp));
    HIP_TRY(c->alloc(&b.stop, (size_t)(params->m1_cgls + 2) * N));
    HIP_TRY(c->alloc(&c->Q, c->nsino));
    if (params->m2_jacobi > 1) {
        HIP_TRY(c->alloc(&c->ua, c->nimg));
        HIP_TRY(c->alloc(&c->ub, c->nimg));
    }
    c->nrelblk = reg_blocks(c->rs);
    HIP_TRY(c->alloc(&c->relpart, 2 * (size_t)c->nrelblk));
    HIP_TRY(c->alloc(&c->flags, 4));
    HIP_TRY(c->alloc(&c->hist, (size_t)params->max_outer));
    HIP_TRY(hipMemset(c->flags, 0, 4 * sizeof(int)));
    HIP_TRY(hipDeviceSynchronize());
    *out = guard.release();
    return TNLM_OK;
}

extern "C" void tnlm_destroy(tnlm_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
}

enum {
    K_PROJECT = TNLM_KIND_PROJECT,
    K_BACKPROJECT = TNLM_KIND_BACKPROJECT,
    K_REGULARIZE = TNLM_KIND_REGULARIZE,
    K_VECTOR = TNLM_KIND_VECTOR,
    K_FBP = TNLM_KIND_FBP,
    K_OTHER = TNLM_KIND_OTHER
};

#define TIMED(c, kind, expr) \
    do {                         \
        (c)->tbegin(kind);       \
        expr;                    \
        (c)->tend();             \
    } while (0)

// ---- data step: u <- CGLS_M1(f) (or Eq. 4), reading y, sw (= sqrt w) / w
static void enqueue_data_step(tnlm_ctx *c, const float *y, const float *w, const float *f, const int *skip) {
    const DevGeom &g = c->dg;
    CglsBufs &b = c->cb;
    hipStream_t st = c->stream;
    const int M1 = c->prm.m1_cgls;
    if (M1 == 0) {
        TIMED(c, K_PROJECT, launch_project(g, PROJ_PLAIN, f, nullptr, nullptr, b.q, nullptr, nullptr, skip, st));
        TIMED(c, K_VECTOR, launch_weighted_resid(g, b.q, y, w, c->Q, skip, st));
        TIMED(c, K_BACKPROJECT, launch_backproject(g, c->Q, b.t, nullptr, skip, st));
        TIMED(c, K_VECTOR, launch_gradient_step(g, f, b.t, 1.0f / c->prm.beta, b.u, skip, st));
        return;
    }
    TIMED(c, K_VECTOR, launch_copy(f, b.u, c->nimg, skip, st));
    TIMED(c, K_PROJECT, launch_project(g, PROJ_RESID, b.u, y, b.sw, b.r, b.rw, nullptr, skip, st));  // r0, sw r0
    TIMED(c, K_BACKPROJECT, launch_backproject(g, b.rw, b.s, b.gpart[0], skip, st));  // s0, ||s0||^2
    for (int m = 0; m < M1; ++m) {
        TIMED(c, K_PROJECT, launch_project(g, PROJ_SCALED, b.s, nullptr, b.sw, b.q, nullptr, b.qpart, skip, st));
        TIMED(c, K_VECTOR, launch_cgls_update(g, b, m, m & 1, skip, st));
        if (m + 1 < M1) {
            TIMED(c, K_BACKPROJECT, launch_backproject(g, b.rw, b.t, b.gpart[(m + 1) & 1], skip, st));
            TIMED(c, K_VECTOR, launch_cgls_direction(g, b, m, m & 1, (m + 1) & 1, skip, st));
        }
    }
}

// ---- Gauss-Jacobi sweeps from g = u, weights from u; last sweep writes f (clamped)
static void enqueue_regularize(tnlm_ctx *c, float *f, const int *skip, bool record) {
    const float *g = c->cb.u;
    const int M2 = c->prm.m2_jacobi;
    const float *val = g;
    for (int m = 0; m < M2; ++m) {
        const bool last = m + 1 == M2;
        float *dst = last ? f : ((m & 1) ? c->ub : c->ua);
        TIMED(c, K_REGULARIZE, launch_regularize(c->rs, g, val, g, dst, last ? 1 : 0, last && record ? c->relpart : nullptr,
                          c->nonfinite(), skip, c->stream));
        val = dst;
    }
}

static void enqueue_step(tnlm_ctx *c, const float *y, const float *w, float *f, const int *skip) {
    enqueue_data_step(c, y, w, f, skip);
    enqueue_regularize(c, f, skip, true);
    TIMED(c, K_OTHER, launch_finalize(c->relpart, c->nrelblk, c->prm.tol_rel_update, c->hist, c->counter(), c->done(),
                    c->nonfinite(), c->prm.max_outer, skip, c->stream));
}

#define CHECK_CTX()                                                                    \
    do {                                                                               \
        if (!ctx) return fail(TNLM_E_INVALID_ARG, "null context");                     \
    } while (0)

#define CHECK_LAUNCH()                                                                 \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess) return fail(TNLM_E_HIP, hipGetErrorString(e_));          \
    } while (0)

extern "C" tnlm_status tnlm_step(tnlm_ctx *ctx, const float *d_y, const float *d_w, float *d_f) {
    CHECK_CTX();
    if (!d_y || !d_w || !d_f) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    if (ctx->prm.m1_cgls > 0) TIMED(ctx, K_VECTOR, launch_sqrt(d_w, ctx->cb.sw, ctx->nsino, ctx->stream));
    enqueue_step(ctx, d_y, d_w, d_f, ctx->zero());
    CHECK_LAUNCH();
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_solve(tnlm_ctx *ctx, const float *d_y, const float *d_w, float *d_f, int32_t *out_iters,
                                  float *out_rel) {
    CHECK_CTX();
    if (!d_y || !d_w || !d_f) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    hipStream_t st = ctx->stream;
    HIP_TRY(hipMemsetAsync(ctx->flags, 0, 4 * sizeof(int), st));
    TIMED(ctx, K_OTHER, launch_check_finite(d_y, ctx->nsino, ctx->nonfinite(), st));
    TIMED(ctx, K_OTHER, launch_check_finite(d_w, ctx->nsino, ctx->nonfinite(), st));
    if (ctx->prm.init == TNLM_INIT_FBP_ALL)
        TIMED(ctx, K_FBP, launch_fbp(ctx->dg, d_y, ctx->hfilt, ctx->cw, ctx->Q, d_f, 1, (float)ctx->geom.sad_mm, st));
    else
        TIMED(ctx, K_OTHER, launch_check_finite(d_f, ctx->nimg, ctx->nonfinite(), st));
    int host_flags[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(host_flags, ctx->flags, sizeof(host_flags), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (host_flags[3]) return fail(TNLM_E_NONFINITE, "non-finite value in y, w or the initial image");
    if (ctx->prm.m1_cgls > 0) TIMED(ctx, K_VECTOR, launch_sqrt(d_w, ctx->cb.sw, ctx->nsino, st));
    const int K = ctx->prm.max_outer;
    const bool early = ctx->prm.tol_rel_update > 0.0f;
    const int chunk = 8;
    for (int k = 0; k < K; ++k) {
        enqueue_step(ctx, d_y, d_w, d_f, ctx->done());
        if (early && ((k + 1) % chunk == 0) && k + 1 < K) {
            HIP_TRY(hipMemcpyAsync(host_flags, ctx->flags, sizeof(host_flags), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (host_flags[1]) break;
        }
    }
    CHECK_LAUNCH();
    HIP_TRY(hipMemcpyAsync(host_flags, ctx->flags, sizeof(host_flags), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int iters = host_flags[2];
    float rel = 0.0f;
    if (iters > 0) HIP_TRY(hipMemcpy(&rel, ctx->hist + (iters - 1), sizeof(float), hipMemcpyDeviceToHost));
    if (out_iters) *out_iters = iters;
    if (out_rel) *out_rel = rel;
    if (host_flags[3]) return fail(TNLM_E_NONFINITE, "an iterate became non-finite");
    if (early && !(rel < ctx->prm.tol_rel_update)) {
        g_last_error = "max_outer reached before tol_rel_update";
        return TNLM_W_NOT_CONVERGED;
    }
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_get_history(tnlm_ctx *ctx, float *out, int32_t n, int32_t *out_n) {
    CHECK_CTX();
    int cnt = 0;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipMemcpy(&cnt, ctx->counter(), sizeof(int), hipMemcpyDeviceToHost));
    cnt = std::min(cnt, ctx->prm.max_outer);
    if (out && n > 0) HIP_TRY(hipMemcpy(out, ctx->hist, sizeof(float) * std::min(n, cnt), hipMemcpyDeviceToHost));
    if (out_n) *out_n = cnt;
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_project(tnlm_ctx *ctx, const float *d_f, float *d_q) {
    CHECK_CTX();
    if (!d_f || !d_q) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    TIMED(ctx, K_PROJECT, launch_project(ctx->dg, PROJ_PLAIN, d_f, nullptr, nullptr, d_q, nullptr, nullptr, nullptr, ctx->stream));
    CHECK_LAUNCH();
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_backproject(tnlm_ctx *ctx, const float *d_q, float *d_f) {
    CHECK_CTX();
    if (!d_f || !d_q) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    TIMED(ctx, K_BACKPROJECT, launch_backproject(ctx->dg, d_q, d_f, nullptr, nullptr, ctx->stream));
    CHECK_LAUNCH();
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_fbp(tnlm_ctx *ctx, const float *d_y, float *d_f, int32_t all_phases) {
    CHECK_CTX();
    if (!d_y || !d_f) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    TIMED(ctx, K_FBP, launch_fbp(ctx->dg, d_y, ctx->hfilt, ctx->cw, ctx->Q, d_f, all_phases ? 1 : 0, (float)ctx->geom.sad_mm,
               ctx->stream));
    CHECK_LAUNCH();
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_data_step(tnlm_ctx *ctx, const float *d_y, const float *d_w, const float *d_f, float *d_g) {
    CHECK_CTX();
    if (!d_y || !d_w || !d_f || !d_g) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    if (d_f == d_g) return fail(TNLM_E_INVALID_ARG, "d_f and d_g must not alias");
    if (ctx->prm.m1_cgls > 0) TIMED(ctx, K_VECTOR, launch_sqrt(d_w, ctx->cb.sw, ctx->nsino, ctx->stream));
    enqueue_data_step(ctx, d_y, d_w, d_f, ctx->zero());
    TIMED(ctx, K_VECTOR, launch_copy(ctx->cb.u, d_g, ctx->nimg, ctx->zero(), ctx->stream));
    CHECK_LAUNCH();
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_regularize(tnlm_ctx *ctx, const float *d_guide, const float *d_value, const float *d_g,
                                       float *d_out, int32_t clamp) {
    CHECK_CTX();
    if (!d_guide || !d_value || !d_g || !d_out) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    if (d_out == d_guide || d_out == d_value || d_out == d_g)
        return fail(TNLM_E_INVALID_ARG, "d_out must not alias an input");
    TIMED(ctx, K_REGULARIZE, launch_regularize(ctx->rs, d_guide, d_value, d_g, d_out, clamp ? 1 : 0, nullptr, nullptr, nullptr, ctx->stream));
    CHECK_LAUNCH();
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_timing_enable(tnlm_ctx *ctx, int32_t enable) {
    CHECK_CTX();
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (auto &r : ctx->recs) {
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    ctx->timing = enable != 0;
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_timing_read(tnlm_ctx *ctx, double *ms, int32_t *launches) {
    CHECK_CTX();
    if (!ms || !launches) return fail(TNLM_E_INVALID_ARG, "null output array");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < TNLM_KIND_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &r : ctx->recs) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.kind] += t;
        launches[r.kind] += 1;
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    return TNLM_OK;
}

extern "C" const char *tnlm_status_string(tnlm_status s) {
    switch (s) {
        case TNLM_OK: return "ok";
        case TNLM_E_INVALID_ARG: return "invalid argument";
        case TNLM_E_SHAPE: return "inconsistent shape";
        case TNLM_E_HIP: return "HIP runtime error";
        case TNLM_E_OOM: return "out of device memory";
        case TNLM_E_NONFINITE: return "non-finite value";
        case TNLM_W_NOT_CONVERGED: return "not converged (max_outer reached)";
    }
    return "unknown status";
}

extern "C" const char *tnlm_last_error(void) { return g_last_error.c_str(); }
