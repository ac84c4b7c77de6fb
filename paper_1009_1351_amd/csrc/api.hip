// Host side of the C ABI declared in include/tnlm.h: argument validation,
// geometry tables, the ragged slice table, scratch ownership, and the enqueue
// order of one outer iteration of the TNLM algorithm box (§2.2), optionally
// captured once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <filesystem>
#include <fstream>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
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

constexpr int kCUs = 256;

}  // namespace

enum {
    K_PROJECT = TNLM_KIND_PROJECT,
    K_BACKPROJECT = TNLM_KIND_BACKPROJECT,
    K_REGULARIZE = TNLM_KIND_REGULARIZE,
    K_VECTOR = TNLM_KIND_VECTOR,
    K_FBP = TNLM_KIND_FBP,
    K_OTHER = TNLM_KIND_OTHER
};

// Everything one batch of slices needs on the device; a single-slice context
// is a batch of one.
struct Engine {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    tnlm_params prm{};
    int ns = 0;
    std::vector<tnlm_geometry> geoms;
    std::vector<std::vector<double>> angles;
    std::vector<SliceDesc> sl;
    std::vector<void *> allocs;
    Batch batch{};
    SliceDesc *d_sl = nullptr;
    float4 *rt0 = nullptr, *vt = nullptr;
    int4 *vo = nullptr;
    float *hfilt = nullptr, *cw = nullptr;
    Stage st_fp{}, st_bp{}, st_vec{}, st_reg{}, st_ffilt{}, st_fbp_all{}, st_fbp_ph{}, st_tr{};
    float *fP = nullptr, *fTP = nullptr;   // padded row-major and transposed copies a projection reads
    size_t npimg = 0;                       // elements of each padded copy
    const float *fixed_guide = nullptr;   // caller's weight guide for every iteration (null: g^(k))
    struct StageSpec {
        Stage *st;
        std::vector<int> counts;
        std::vector<double> cost;
        int *pre, *xb;   // device tables of st
    };
    std::vector<StageSpec> specs;
    std::vector<int> restage_buf;   // host staging of the re-cut tables
    CglsBufs cb{};
    float *Q = nullptr, *ua = nullptr, *ub = nullptr;
    double *relpart = nullptr;
    float2 *symfwd = nullptr;   // symmetric-reuse regulariser: forward sums per image element
    float2 *sympart = nullptr;  // and reverse partial sums (image-shaped planes)
    double *cost_part = nullptr;   // [1024] partials of the data-term reduction
    int *flags = nullptr;   // [4][ns]: done, counter, nonfinite, spare
    int *queue = nullptr;   // [16]: work-item counters of the persistent stages (cleared by each launch)
    float *hist = nullptr;  // [ns][max_outer]
    float *Y = nullptr, *Wt = nullptr, *F = nullptr;   // batch copies of caller arrays
    size_t nimg = 0, nsino = 0;
    int rows_per_lane = 8;
    RegParams rp{};
    // graph of one outer iteration for a given (y, w, f)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void *gkey[3] = {nullptr, nullptr, nullptr};
    bool use_graph = true;

    // kernel timing (HIP events around every launch)
    struct TimedRec {
        int kind;
        hipEvent_t a, b;
    };
    bool timing = false;
    std::vector<TimedRec> recs;
    std::vector<hipEvent_t> pool;
    TimedRec pending{};
    hipStream_t cur = nullptr;   // stream the enqueue functions target

    int *done() { return flags; }
    int *counter() { return flags + ns; }
    int *nonfinite() { return flags + 2 * ns; }

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
        (void)hipEventRecord(pending.a, cur);
    }
    void tend() {
        if (!timing) return;
        (void)hipEventRecord(pending.b, cur);
        recs.push_back(pending);
    }
    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        gkey[0] = gkey[1] = gkey[2] = nullptr;
    }
    ~Engine() {
        (void)hipStreamSynchronize(stream);
        drop_graph();
        for (auto &r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        for (void *p : allocs) (void)hipFree(p);
    }
};

struct tnlm_ctx {
    Engine e;
};
struct tnlm_batch {
    Engine e;
};

#define TIMED(E, kind, expr) \
    do {                     \
        (E)->tbegin(kind);   \
        expr;                \
        (E)->tend();         \
    } while (0)

// ---------------------------------------------------------------------------
// validation and tables
// ---------------------------------------------------------------------------
static tnlm_status validate_geom(const tnlm_geometry *g) {
    if (!g) return fail(TNLM_E_INVALID_ARG, "null geometry");
    if (g->n_phases < 1 || g->L < 1 || g->L > 4096 || g->n_views < 1 || g->n_bins < 1 || g->n_bins > 4096)
        return fail(TNLM_E_SHAPE, "need N >= 1, 1 <= L <= 4096, V >= 1, 1 <= B <= 4096");
    if ((long long)g->n_phases * g->n_views * g->n_bins > (1LL << 31) ||
        (long long)g->n_phases * g->L * g->L > (1LL << 31))
        return fail(TNLM_E_SHAPE, "slice too large");
    if (!(g->pixel_mm > 0) || !(g->sad_mm > 0) || !(g->dgamma_rad > 0) || !g->view_angles_rad)
        return fail(TNLM_E_INVALID_ARG, "need pixel_mm, sad_mm, dgamma_rad > 0 and view angles");
    if (!std::isfinite(g->det_offset_bins)) return fail(TNLM_E_INVALID_ARG, "det_offset_bins not finite");
    const double half_diag = 0.7071067811865476 * g->pixel_mm * g->L;
    if (!(g->sad_mm > half_diag + 2.0 * g->pixel_mm))
        return fail(TNLM_E_INVALID_ARG, "the source circle must enclose the image square (SAD > half-diagonal + 2 pixels)");
    if (!((g->n_bins - 1) * g->dgamma_rad < M_PI)) return fail(TNLM_E_INVALID_ARG, "the fan must be narrower than pi");
    for (long k = 0; k < (long)g->n_phases * g->n_views; ++k)
        if (!std::isfinite(g->view_angles_rad[k])) return fail(TNLM_E_NONFINITE, "non-finite view angle");
    return TNLM_OK;
}

static tnlm_status validate_params(const tnlm_params *p, int minL) {
    if (!p) return fail(TNLM_E_INVALID_ARG, "null params");
    if (!(p->patch & 1) || !(p->window & 1) || !reg_supported(p->patch, p->window))
        return fail(TNLM_E_INVALID_ARG, "patch must be odd in [3,9], window odd in [3,21]");
    if (p->window > minL) return fail(TNLM_E_SHAPE, "window larger than the image");
    if (!(p->h > 0) || !std::isfinite(p->h)) return fail(TNLM_E_INVALID_ARG, "h must be > 0");
    if (!(p->mu_hat >= 0) || !std::isfinite(p->mu_hat)) return fail(TNLM_E_INVALID_ARG, "mu_hat must be >= 0");
    if (!(p->beta > 0) || !std::isfinite(p->beta)) return fail(TNLM_E_INVALID_ARG, "beta must be > 0");
    if (p->m1_cgls < 0 || p->m1_cgls > 64) return fail(TNLM_E_INVALID_ARG, "m1_cgls must be in [0, 64]");
    if (p->m2_jacobi < 1 || p->m2_jacobi > 1000) return fail(TNLM_E_INVALID_ARG, "m2_jacobi must be in [1, 1000]");
    if (p->max_outer < 1 || p->max_outer > 100000) return fail(TNLM_E_INVALID_ARG, "max_outer must be >= 1");
    if (!(p->tol_rel_update >= 0)) return fail(TNLM_E_INVALID_ARG, "tol_rel_update must be >= 0");
    if (p->init != TNLM_INIT_FBP_ALL && p->init != TNLM_INIT_USER) return fail(TNLM_E_INVALID_ARG, "bad init");
    if (p->ssd_mode != TNLM_SSD_FP32 && p->ssd_mode != TNLM_SSD_BF16_MFMA && p->ssd_mode != TNLM_SSD_FP32_SYMMETRIC)
        return fail(TNLM_E_INVALID_ARG, "bad ssd_mode");
    if (p->ssd_mode == TNLM_SSD_FP32_SYMMETRIC && !reg_sym_supported(p->patch, p->window))
        return fail(TNLM_E_INVALID_ARG, "ssd_mode FP32_SYMMETRIC: patch and window need more LDS than a block has");
    if (p->ssd_mode == TNLM_SSD_BF16_MFMA && !reg_mfma_supported(p->patch, p->window))
        return fail(TNLM_E_INVALID_ARG, "ssd_mode BF16_MFMA supports patch 3, 5, 7 and window <= 15");
    return TNLM_OK;
}

// Per-ray plane tables in double precision, rounded once to float.
// crossings receives the slice's ray-pixel crossings (|dc| + |dr| + 1 cells
// per ray that meets the image), the cost of one forward projection.
static bool append_tables(const tnlm_geometry &g, std::vector<float4> &rt0, std::vector<float4> &vt,
                          std::vector<int4> &vo, std::vector<float> &hf, std::vector<float> &cw, double &crossings) {
    crossings = 0.0;
    const int N = g.n_phases, V = g.n_views, B = g.n_bins, L = g.L;
    const double D = g.pixel_mm, X0 = -0.5 * D * L;
    for (int i = 0; i < N; ++i)
        for (int v = 0; v < V; ++v) {
            const double th = g.view_angles_rad[(size_t)i * V + v];
            const double sx = g.sad_mm * std::cos(th), sy = g.sad_mm * std::sin(th);
            vt.push_back(make_float4((float)sx, (float)sy, (float)std::cos(th), (float)std::sin(th)));
            for (int b = 0; b < B; ++b) {
                const double gam = ((double)b - 0.5 * (B - 1) + g.det_offset_bins) * g.dgamma_rad;
                const double ux = std::cos(th + M_PI + gam), uy = std::sin(th + M_PI + gam);
                const double ts = -(sx * ux + sy * uy);   // source -> point nearest the centre
                const double ox = sx + ts * ux, oy = sy + ts * uy;
                const double ix = std::fabs(ux) > 1e-9 ? 1.0 / ux : std::copysign(1e9, ux == 0 ? 1.0 : ux);
                const double iy = std::fabs(uy) > 1e-9 ? 1.0 / uy : std::copysign(1e9, uy == 0 ? 1.0 : uy);
                rt0.push_back(make_float4((float)(D * ix), (float)((X0 - ox) * ix), (float)(D * iy),
                                          (float)((X0 - oy) * iy)));
                const double ax = (X0 - ox) * ix, bxp = (X0 + D * L - ox) * ix;
                const double ay = (X0 - oy) * iy, byp = (X0 + D * L - oy) * iy;
                const double chord = std::min(std::max(ax, bxp), std::max(ay, byp)) -
                                     std::max(std::min(ax, bxp), std::min(ay, byp));
                if (chord > 0.0) crossings += chord * (std::fabs(ux) + std::fabs(uy)) / D + 1.0;
            }
            // orientation of the view's rays: the sign of Ax (and Ay) is that of
            // bin 0 below bin bx (by) and the opposite from there on; the fan is
            // narrower than pi, so each sign changes at most once across it
            const float4 *r = rt0.data() + rt0.size() - B;
            const bool x0 = r[0].x > 0.0f, y0 = r[0].z > 0.0f;
            int bx = B, by = B;
            for (int b = B - 1; b >= 0; --b) {
                if ((r[b].x > 0.0f) != x0) bx = b;
                if ((r[b].z > 0.0f) != y0) by = b;
            }
            for (int b = 0; b < B; ++b)   // the back-projector relies on a single change
                if (((r[b].x > 0.0f) != x0) != (b >= bx) || ((r[b].z > 0.0f) != y0) != (b >= by)) return false;
            vo.push_back(make_int4(bx, by, (x0 ? 1 : 0) | (y0 ? 2 : 0), 0));
        }
    const double a = g.dgamma_rad;
    for (int m = -(B - 1); m <= B - 1; ++m) {
        double h;
        if (m == 0) h = 1.0 / (8.0 * a * a);
        else if (m % 2 == 0) h = 0.0;
        else {
            const double s = std::sin(m * a);
            h = -1.0 / (2.0 * M_PI * M_PI * s * s);
        }
        hf.push_back((float)(a * h));
    }
    for (int b = 0; b < B; ++b)
        cw.push_back((float)(g.sad_mm * std::cos(((double)b - 0.5 * (B - 1) + g.det_offset_bins) * a)));
    return true;
}

// Work items of a stage: counts[s] items of slice s, each of estimated cost
// cost[s] (empty: all equal); slices with active[s] == 0 get no items.
// Besides the prefix table (pre, ns + 1 entries), the item boundaries of the
// 8 XCD ranges (xb, 9 entries) are cut at equal cumulative cost.
static void stage_tables(const std::vector<int> &counts, const std::vector<double> &cost,
                         const std::vector<char> &active, int *pre, int *xb) {
    const size_t ns = counts.size();
    std::vector<double> cpre(ns + 1, 0.0);
    pre[0] = 0;
    for (size_t s = 0; s < ns; ++s) {
        const int n = active.empty() || active[s] ? counts[s] : 0;
        pre[s + 1] = pre[s] + n;
        cpre[s + 1] = cpre[s] + n * (cost.empty() ? 1.0 : cost[s]);
    }
    xb[0] = 0;
    for (int x = 1; x < 8; ++x) {
        const double target = cpre[ns] * x / 8.0;
        size_t s = 0;
        while (s + 1 < ns && cpre[s + 1] < target) ++s;
        const double c = cost.empty() ? 1.0 : cost[s];
        const double k = c > 0.0 ? std::ceil((target - cpre[s]) / c) : 0.0;
        xb[x] = std::max(xb[x - 1], std::min(pre[s] + (int)std::max(0.0, k), pre[s + 1]));
    }
    xb[8] = pre[ns];
}

static tnlm_status make_stage(Engine &E, Stage &st, const std::vector<int> &counts, int cap,
                              const std::vector<double> &cost = {}) {
    const size_t ns = counts.size();
    std::vector<int> pre(ns + 1, 0), xb(9, 0);
    stage_tables(counts, cost, {}, pre.data(), xb.data());
    int *d = nullptr, *dx = nullptr;
    HIP_TRY(E.alloc(&d, pre.size()));
    HIP_TRY(hipMemcpy(d, pre.data(), pre.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(E.alloc(&dx, xb.size()));
    HIP_TRY(hipMemcpy(dx, xb.data(), xb.size() * sizeof(int), hipMemcpyHostToDevice));
    st.pre = d;
    st.xb = dx;
    // remembered for re-cutting the tables to the slices still running
    bool found = false;
    for (auto &sp : E.specs)
        if (sp.st == &st) {
            sp = {&st, counts, cost, d, dx};
            found = true;
        }
    if (!found) E.specs.push_back({&st, counts, cost, d, dx});
    st.total = pre.back();
    int g = std::min(st.total, cap);
    if (g >= 8) g -= g % 8;
    st.grid = std::max(1, g);
    return TNLM_OK;
}

static int autotuned_rows_per_lane(const tnlm_params &p, int L);
static tnlm_status engine_autotune(Engine *E, int *chosen, float *ms_out);

static tnlm_status engine_init(Engine &E, int ns, const tnlm_geometry *geoms, const tnlm_params *params,
                               void *stream) {
    if (ns < 1 || !geoms) return fail(TNLM_E_INVALID_ARG, "need at least one slice");
    int minL = 1 << 30;
    for (int s = 0; s < ns; ++s) {
        tnlm_status st = validate_geom(&geoms[s]);
        if (st != TNLM_OK) return st;
        minL = std::min(minL, geoms[s].L);
    }
    tnlm_status st = validate_params(params, minL);
    if (st != TNLM_OK) return st;
    HIP_TRY(hipGetDevice(&E.device));
    E.stream = (hipStream_t)stream;
    E.cur = E.stream;
    E.prm = *params;
    E.ns = ns;
    E.rp = RegParams{params->patch, params->window, params->h, params->mu_hat};
    // tile height: forced by TNLM_ROWS_PER_LANE, else the cached choice for
    // this (patch, window, L) class, else tuned at the end of the set-up
    const char *env_rpl = std::getenv("TNLM_ROWS_PER_LANE");
    const int cached_rpl = env_rpl ? (std::atoi(env_rpl) == 4 ? 4 : 8) : autotuned_rows_per_lane(*params, geoms[0].L);
    E.rows_per_lane = params->ssd_mode == TNLM_SSD_FP32_SYMMETRIC ? reg_sym_rows_per_lane()
                      : cached_rpl                                  ? cached_rpl
                                                                    : 8;
    const bool tune_now = cached_rpl == 0 && params->ssd_mode == TNLM_SSD_FP32;
    const char *env_graph = std::getenv("TNLM_NO_GRAPH");
    E.use_graph = !(env_graph && env_graph[0] == '1');

    std::vector<float4> rt0, vt;
    std::vector<int4> vo;
    std::vector<float> hf, cw;
    E.geoms.assign(geoms, geoms + ns);
    std::vector<double> crossings(ns, 0.0);
    E.angles.resize(ns);
    E.sl.resize(ns);
    long long ray = 0, view = 0, img = 0, sino = 0, pimg = 0;
    int gp = 0, qp = 0, rpp = 0, phase = 0;
    for (int s = 0; s < ns; ++s) {
        const tnlm_geometry &g = geoms[s];
        E.angles[s].assign(g.view_angles_rad, g.view_angles_rad + (size_t)g.n_phases * g.n_views);
        E.geoms[s].view_angles_rad = E.angles[s].data();
        SliceDesc &d = E.sl[s];
        d.N = g.n_phases;
        d.L = g.L;
        d.V = g.n_views;
        d.B = g.n_bins;
        d.D = (float)g.pixel_mm;
        d.X0 = (float)(-0.5 * g.pixel_mm * g.L);
        d.dgamma = (float)g.dgamma_rad;
        d.ucenter = (float)(0.5 * (g.n_bins - 1) - g.det_offset_bins);
        d.ray0 = ray;
        d.view0 = view;
        d.img0 = img;
        d.pimg0 = pimg;
        d.sino0 = sino;
        d.hf0 = (int)hf.size();
        d.cw0 = (int)cw.size();
        if (!append_tables(E.geoms[s], rt0, vt, vo, hf, cw, crossings[s]))
            return fail(TNLM_E_INVALID_ARG, "ray directions change sign more than once across the fan");
        d.nbp = bp_blocks(d) / d.N;
        d.npp = proj_blocks(d) / d.N;
        d.nrb = params->ssd_mode == TNLM_SSD_BF16_MFMA ? reg_mfma_blocks(d)
                                                       : reg_blocks(d, params->patch, E.rows_per_lane);
        d.gp0 = gp;
        d.qp0 = qp;
        d.rp0 = rpp;
        d.phase0 = phase;
        gp += d.N * d.nbp;
        qp += d.N * d.npp;
        rpp += d.nrb;
        phase += d.N;
        ray += (long long)d.N * d.V * d.B;
        view += (long long)d.N * d.V;
        img += (long long)d.N * d.L * d.L;
        pimg += (long long)d.N * d.L * (d.L + 2);
        sino += (long long)d.N * d.V * d.B;
    }
    E.nimg = (size_t)img;
    E.npimg = (size_t)pimg;
    E.nsino = (size_t)sino;
    HIP_TRY(E.alloc(&E.d_sl, ns));
    HIP_TRY(hipMemcpy(E.d_sl, E.sl.data(), ns * sizeof(SliceDesc), hipMemcpyHostToDevice));
    HIP_TRY(E.alloc(&E.rt0, rt0.size()));
    HIP_TRY(E.alloc(&E.vt, vt.size()));
    HIP_TRY(E.alloc(&E.vo, vo.size()));
    HIP_TRY(E.alloc(&E.hfilt, hf.size()));
    HIP_TRY(E.alloc(&E.cw, cw.size()));
    HIP_TRY(hipMemcpy(E.rt0, rt0.data(), rt0.size() * sizeof(float4), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(E.vt, vt.data(), vt.size() * sizeof(float4), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(E.vo, vo.data(), vo.size() * sizeof(int4), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(E.hfilt, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(E.cw, cw.data(), cw.size() * sizeof(float), hipMemcpyHostToDevice));
    E.batch.ns = ns;
    E.batch.sl = E.d_sl;
    E.batch.rt0 = E.rt0;
    E.batch.vt = E.vt;
    E.batch.vo = E.vo;
    E.batch.skip = nullptr;

    std::vector<int> cfp, cbp, cvec, creg, cff, cfa, cfph, ctr;
    std::vector<double> kfp, kbp;
    for (auto &d : E.sl) {
        cfp.push_back(proj_blocks(d));
        cbp.push_back(bp_blocks(d));
        ctr.push_back(tr_blocks(d));
        // cost models: a projector block walks its rays' crossings (the
        // slice's crossings over its blocks: ray lengths and the share of a
        // slice's last bin block that holds rays differ between slices); a
        // back-projector tile runs V views of a ~40-operation set-up plus
        // ~14 operations per candidate bin, ~1.5 + D / (dgamma * SAD) bins
        const size_t si = (size_t)(&d - E.sl.data());
        kfp.push_back(crossings[si] / std::max(1, proj_blocks(d)));
        const double cand = 1.5 + (double)d.D / ((double)d.dgamma * E.geoms[si].sad_mm);
        kbp.push_back(d.V * (40.0 + 14.0 * cand));
        cvec.push_back(d.N * vec_blocks(d));
        creg.push_back(d.nrb);
        cff.push_back(d.N * d.V);
        cfa.push_back(fbp_bp_blocks(d, 1));
        cfph.push_back(fbp_bp_blocks(d, 0));
    }
    if ((st = make_stage(E, E.st_fp, cfp, kCUs * 8, kfp)) != TNLM_OK) return st;
    if ((st = make_stage(E, E.st_bp, cbp, kCUs * 8, kbp)) != TNLM_OK) return st;
    E.st_fp.cu_runs = 1;
    E.st_bp.cu_runs = 1;
    E.st_fp.prefetch = 1;   // many short items (one view's 256 rays each)
    // one set of work-item counters serves the persistent stages: their
    // launches are ordered on the engine's stream, and each launch leaves the
    // counters cleared
    HIP_TRY(E.alloc(&E.queue, 16));
    HIP_TRY(hipMemset(E.queue, 0, 16 * sizeof(int)));
    E.st_fp.queue = E.st_bp.queue = E.st_reg.queue = E.queue;
    if ((st = make_stage(E, E.st_vec, cvec, kCUs * 8)) != TNLM_OK) return st;
    if ((st = make_stage(E, E.st_reg, creg, kCUs * 4)) != TNLM_OK) return st;
    if ((st = make_stage(E, E.st_ffilt, cff, kCUs * 8)) != TNLM_OK) return st;
    if ((st = make_stage(E, E.st_fbp_all, cfa, kCUs * 8)) != TNLM_OK) return st;
    if ((st = make_stage(E, E.st_fbp_ph, cfph, kCUs * 8)) != TNLM_OK) return st;
    if ((st = make_stage(E, E.st_tr, ctr, kCUs * 8)) != TNLM_OK) return st;
    HIP_TRY(E.alloc(&E.fP, E.npimg));
    HIP_TRY(E.alloc(&E.fTP, E.npimg));
    // the zero columns of the padded copies; kernels write only the interior
    HIP_TRY(hipMemset(E.fP, 0, E.npimg * sizeof(float)));
    HIP_TRY(hipMemset(E.fTP, 0, E.npimg * sizeof(float)));

    CglsBufs &b = E.cb;
    HIP_TRY(E.alloc(&b.u, E.nimg));
    HIP_TRY(E.alloc(&b.s, E.nimg));
    HIP_TRY(E.alloc(&b.t, E.nimg));
    HIP_TRY(E.alloc(&b.r, E.nsino));
    HIP_TRY(E.alloc(&b.q, E.nsino));
    HIP_TRY(E.alloc(&b.rw, E.nsino));
    HIP_TRY(E.alloc(&b.sw, E.nsino));
    HIP_TRY(E.alloc(&b.gpart[0], (size_t)gp));
    HIP_TRY(E.alloc(&b.gpart[1], (size_t)gp));
    HIP_TRY(E.alloc(&b.qpart, (size_t)qp));
    b.nphase = phase;
    HIP_TRY(E.alloc(&b.stop, (size_t)(params->m1_cgls + 2) * phase));
    HIP_TRY(E.alloc(&E.Q, E.nsino));
    if (params->m2_jacobi > 1) {
        HIP_TRY(E.alloc(&E.ua, E.nimg));
        HIP_TRY(E.alloc(&E.ub, E.nimg));
    }
    HIP_TRY(E.alloc(&E.relpart, 2 * (size_t)rpp));
    if (params->ssd_mode == TNLM_SSD_FP32_SYMMETRIC) {
        HIP_TRY(E.alloc(&E.symfwd, E.nimg));
        HIP_TRY(E.alloc(&E.sympart, (size_t)reg_sym_planes(params->patch, params->window) * E.nimg));
    }
    HIP_TRY(E.alloc(&E.flags, 4 * (size_t)ns));
    HIP_TRY(E.alloc(&E.cost_part, 1024));
    HIP_TRY(E.alloc(&E.hist, (size_t)ns * params->max_outer));
    HIP_TRY(hipMemset(E.flags, 0, 4 * ns * sizeof(int)));
    HIP_TRY(hipStreamCreateWithFlags(&E.capture_stream, hipStreamNonBlocking));
    HIP_TRY(hipDeviceSynchronize());
    if (tune_now) return engine_autotune(&E, nullptr, nullptr);
    return TNLM_OK;
}

// ---------------------------------------------------------------------------
// enqueue order of one outer iteration
// ---------------------------------------------------------------------------
// data step: u <- CGLS_M1(f) (or Eq. 4), reading y, sw = sqrt(w) / w
static void enqueue_data_step(Engine *E, const Batch &bt, const float *y, const float *w, const float *f) {
    CglsBufs &b = E->cb;
    hipStream_t st = E->cur;
    const int M1 = E->prm.m1_cgls;
    if (M1 == 0) {
        TIMED(E, K_VECTOR, launch_transpose(bt, E->st_tr, f, E->fP, E->fTP, st));
        TIMED(E, K_PROJECT,
              launch_project(bt, E->st_fp, PROJ_PLAIN, E->fP, E->fTP, nullptr, nullptr, b.q, nullptr, nullptr, st));
        TIMED(E, K_VECTOR, launch_weighted_resid(bt, E->st_vec, b.q, y, w, E->Q, st));
        TIMED(E, K_BACKPROJECT, launch_backproject(bt, E->st_bp, E->Q, b.t, nullptr, st));
        TIMED(E, K_VECTOR, launch_gradient_step(bt, E->st_vec, f, b.t, 1.0f / E->prm.beta, b.u, st));
        return;
    }
    TIMED(E, K_VECTOR, launch_copy_skip(bt, E->st_vec, true, f, b.u, st));
    TIMED(E, K_VECTOR, launch_transpose(bt, E->st_tr, b.u, E->fP, E->fTP, st));
    TIMED(E, K_PROJECT, launch_project(bt, E->st_fp, PROJ_RESID, E->fP, E->fTP, y, b.sw, b.r, b.rw, nullptr, st));
    TIMED(E, K_BACKPROJECT, launch_backproject(bt, E->st_bp, b.rw, b.s, b.gpart[0], st));
    for (int m = 0; m < M1; ++m) {
        TIMED(E, K_VECTOR, launch_transpose(bt, E->st_tr, b.s, E->fP, E->fTP, st));
        TIMED(E, K_PROJECT,
              launch_project(bt, E->st_fp, PROJ_SCALED, E->fP, E->fTP, nullptr, b.sw, b.q, nullptr, b.qpart, st));
        TIMED(E, K_VECTOR, launch_cgls_update(bt, E->st_vec, b, m, m & 1, st));
        if (m + 1 < M1) {
            TIMED(E, K_BACKPROJECT, launch_backproject(bt, E->st_bp, b.rw, b.t, b.gpart[(m + 1) & 1], st));
            TIMED(E, K_VECTOR, launch_cgls_direction(bt, E->st_vec, b, m, m & 1, (m + 1) & 1, st));
        }
    }
}

// Gauss-Jacobi sweeps from g = u, weights from u; last sweep writes f (clamped)
static void enqueue_regularize(Engine *E, const Batch &bt, float *f, bool record) {
    const float *g = E->cb.u;
    const float *guide = E->fixed_guide ? E->fixed_guide : g;
    const int M2 = E->prm.m2_jacobi;
    const float *val = g;
    for (int m = 0; m < M2; ++m) {
        const bool last = m + 1 == M2;
        float *dst = last ? f : ((m & 1) ? E->ub : E->ua);
        if (E->prm.ssd_mode == TNLM_SSD_BF16_MFMA)
            TIMED(E, K_REGULARIZE,
                  launch_regularize_mfma(bt, E->st_reg, E->rp, guide, val, g, dst, last ? 1 : 0,
                                         last && record ? E->relpart : nullptr, E->nonfinite(), E->cur));
        else if (E->prm.ssd_mode == TNLM_SSD_FP32_SYMMETRIC)
            TIMED(E, K_REGULARIZE,
                  launch_regularize_sym(bt, E->st_reg, E->rp, guide, val, g, dst, last ? 1 : 0,
                                        last && record ? E->relpart : nullptr, E->nonfinite(), E->symfwd,
                                        E->sympart, E->nimg, E->cur));
        else
            TIMED(E, K_REGULARIZE,
                  launch_regularize(bt, E->st_reg, E->rp, E->rows_per_lane, guide, val, g, dst, last ? 1 : 0,
                                    last && record ? E->relpart : nullptr, E->nonfinite(), E->cur));
        val = dst;
    }
}

static void enqueue_step(Engine *E, const Batch &bt, const float *y, const float *w, float *f) {
    enqueue_data_step(E, bt, y, w, f);
    enqueue_regularize(E, bt, f, true);
    TIMED(E, K_OTHER, launch_finalize(bt, E->relpart, E->prm.tol_rel_update, E->hist, E->counter(), E->done(),
                                      E->nonfinite(), E->prm.max_outer, E->cur));
}

static tnlm_status last_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TNLM_E_HIP, hipGetErrorString(e));
    return TNLM_OK;
}

// Graph of one outer iteration with the solve's skip flags, for (y, w, f).
static bool ensure_graph(Engine *E, const Batch &bt, const float *y, const float *w, float *f) {
    if (!E->use_graph || E->timing) return false;
    if (E->gexec && E->gkey[0] == y && E->gkey[1] == w && E->gkey[2] == f) return true;
    E->drop_graph();
    if (hipStreamBeginCapture(E->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    E->cur = E->capture_stream;
    enqueue_step(E, bt, y, w, f);
    E->cur = E->stream;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(E->capture_stream, &g) != hipSuccess || !g) {
        (void)hipGetLastError();
        return false;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(g);
        return false;
    }
    E->graph = g;
    E->gexec = ex;
    E->gkey[0] = y;
    E->gkey[1] = w;
    E->gkey[2] = f;
    return true;
}

// Re-cut every stage's work tables to the slices with active[s] != 0 (empty:
// all). Asynchronous on the engine stream, ordered before the next launch; the
// launches (and a captured graph) keep their configuration.
static tnlm_status restage(Engine *E, const std::vector<char> &active) {
    const size_t ns = (size_t)E->ns;
    HIP_TRY(hipStreamSynchronize(E->stream));   // the previous tables have been copied
    E->restage_buf.assign(E->specs.size() * (ns + 1 + 9), 0);
    for (size_t k = 0; k < E->specs.size(); ++k) {
        auto &sp = E->specs[k];
        int *pre = E->restage_buf.data() + k * (ns + 10), *xb = pre + ns + 1;
        stage_tables(sp.counts, sp.cost, active, pre, xb);
        HIP_TRY(hipMemcpyAsync(sp.pre, pre, (ns + 1) * sizeof(int), hipMemcpyHostToDevice, E->stream));
        HIP_TRY(hipMemcpyAsync(sp.xb, xb, 9 * sizeof(int), hipMemcpyHostToDevice, E->stream));
    }
    return TNLM_OK;
}

// Full solve on contiguous batch arrays (y, w, f); f holds f^(0) when init is user.
// active (nullable, [ns]): slices with 0 take no part (marked finished from
// the start and left out of the work tables; their images are not written)
static tnlm_status engine_solve(Engine *E, const float *y, const float *w, float *f,
                                const std::vector<char> *active = nullptr) {
    hipStream_t st = E->stream;
    E->cur = st;
    const int ns = E->ns;
    Batch bt = E->batch;
    launch_fill_int(E->flags, 4 * ns, 0, st);
    int ninactive = 0;
    if (active) {
        std::vector<int> dn(ns);
        for (int s = 0; s < ns; ++s) ninactive += (dn[s] = (*active)[s] ? 0 : 1);
        HIP_TRY(hipMemcpyAsync(E->done(), dn.data(), ns * sizeof(int), hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));   // dn leaves scope
    }
    if (!active) {
        TIMED(E, K_OTHER, launch_check_finite(y, E->nsino, E->nonfinite(), st));
        TIMED(E, K_OTHER, launch_check_finite(w, E->nsino, E->nonfinite(), st));
    } else {   // only the active slices' data (the others' regions may hold anything)
        for (int s = 0; s < ns; ++s) {
            if (!(*active)[s]) continue;
            const SliceDesc &d = E->sl[s];
            const size_t nsn = (size_t)d.N * d.V * d.B;
            TIMED(E, K_OTHER, launch_check_finite(y + d.sino0, nsn, E->nonfinite(), st));
            TIMED(E, K_OTHER, launch_check_finite(w + d.sino0, nsn, E->nonfinite(), st));
            if (E->prm.init != TNLM_INIT_FBP_ALL)
                TIMED(E, K_OTHER, launch_check_finite(f + d.img0, (size_t)d.N * d.L * d.L, E->nonfinite(), st));
        }
    }
    if (E->prm.init == TNLM_INIT_FBP_ALL)
        TIMED(E, K_FBP, launch_fbp(bt, E->st_ffilt, E->st_fbp_all, y, E->hfilt, E->cw, E->Q, f, 1, st));
    else if (!active)
        TIMED(E, K_OTHER, launch_check_finite(f, E->nimg, E->nonfinite(), st));
    if (E->prm.m1_cgls > 0) TIMED(E, K_VECTOR, launch_sqrt(w, E->cb.sw, E->nsino, st));
    std::vector<int> hf(4 * ns, 0);
    HIP_TRY(hipMemcpyAsync(hf.data(), E->flags, hf.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int s = 0; s < ns; ++s)
        if (hf[2 * ns + s])
            return fail(TNLM_E_NONFINITE, "non-finite value in y, w or the initial image of slice " + std::to_string(s));
    // converged (or failed) slices drop out: every iteration kernel skips them
    bt.skip = E->done();
    const bool graph = ensure_graph(E, bt, y, w, f);
    const int K = E->prm.max_outer;
    const bool early = E->prm.tol_rel_update > 0.0f;
    const int chunk = 8;
    int ndone = 0;   // slices the work tables currently leave out
    tnlm_status rs = TNLM_OK;
    if (ninactive == ns) return TNLM_OK;
    if (ninactive > 0 && ns > 1) {
        if ((rs = restage(E, *active)) != TNLM_OK) return rs;
        ndone = ninactive;
    }
    for (int k = 0; k < K; ++k) {
        if (graph) HIP_TRY(hipGraphLaunch(E->gexec, st));
        else enqueue_step(E, bt, y, w, f);
        if (early && ((k + 1) % chunk == 0) && k + 1 < K) {
            HIP_TRY(hipMemcpyAsync(hf.data(), E->flags, ns * sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            int done = 0;
            for (int s = 0; s < ns; ++s) done += hf[s] != 0;
            if (done == ns) break;
            // finished slices keep their skip flags; once a quarter of the
            // slices that were running at the last cut has finished, re-cut
            // the work tables so the remaining ones spread over all XCDs again
            // (measured against the whole batch, the last few slices of a
            // batch ran on the few XCDs whose ranges still held them)
            if (ns > 1 && done > ndone && 4 * (done - ndone) >= ns - ndone) {
                std::vector<char> active(ns);
                for (int s = 0; s < ns; ++s) active[s] = hf[s] == 0;
                if ((rs = restage(E, active)) != TNLM_OK) break;
                ndone = done;
            }
        }
    }
    tnlm_status ls = last_launch();
    if (ls == TNLM_OK && ndone > 0) ls = restage(E, {});   // full tables for the next call
    if (rs != TNLM_OK) return rs;
    if (ls != TNLM_OK) return ls;
    HIP_TRY(hipStreamSynchronize(st));
    return TNLM_OK;
}

// per-slice results after engine_solve
static tnlm_status engine_results(Engine *E, int32_t *iters, float *rel, tnlm_status *status) {
    const int ns = E->ns;
    std::vector<int> hf(4 * ns, 0);
    HIP_TRY(hipMemcpy(hf.data(), E->flags, hf.size() * sizeof(int), hipMemcpyDeviceToHost));
    tnlm_status worst = TNLM_OK;
    for (int s = 0; s < ns; ++s) {
        const int it = std::min(hf[ns + s], E->prm.max_outer);
        float r = 0.0f;
        if (it > 0)
            HIP_TRY(hipMemcpy(&r, E->hist + (size_t)s * E->prm.max_outer + (it - 1), sizeof(float),
                              hipMemcpyDeviceToHost));
        tnlm_status ss = TNLM_OK;
        if (hf[2 * ns + s]) ss = TNLM_E_NONFINITE;
        else if (E->prm.tol_rel_update > 0.0f && !(r < E->prm.tol_rel_update)) ss = TNLM_W_NOT_CONVERGED;
        if (iters) iters[s] = it;
        if (rel) rel[s] = r;
        if (status) status[s] = ss;
        if (ss < 0) worst = ss;
        else if (ss > 0 && worst == TNLM_OK) worst = ss;
    }
    return worst;
}

// ---------------------------------------------------------------------------
// autotuner: rows per lane of the regulariser tile (4 or 8), per (patch,
// window, L class); both candidates are timed on the device and must agree
// bitwise; results are cached as JSON lines (last entry of a key wins).
// ---------------------------------------------------------------------------
static std::string tune_cache_path() {
    const char *p = std::getenv("TNLM_AUTOTUNE_CACHE");
    if (p && *p) return p;
    const char *home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/tnlm_autotune.jsonl";
}

static std::string tune_key(const tnlm_params &p, int L) {
    int Lc = 64;
    while (Lc < L) Lc *= 2;
    std::ostringstream k;
    k << "gfx950/patch" << p.patch << "/window" << p.window << "/L" << Lc;
    return k.str();
}

static int autotuned_rows_per_lane(const tnlm_params &p, int L) {
    std::ifstream in(tune_cache_path());
    std::string line, key = "\"" + tune_key(p, L) + "\"";
    int v = 0;   // no entry
    while (std::getline(in, line)) {
        if (line.find(key) == std::string::npos) continue;
        const size_t k = line.find("\"rows_per_lane\":");
        if (k != std::string::npos) v = std::atoi(line.c_str() + k + 16) == 4 ? 4 : 8;
    }
    return v;
}

static tnlm_status engine_autotune(Engine *E, int *chosen, float *ms_out) {
    if (E->prm.ssd_mode != TNLM_SSD_FP32) return fail(TNLM_E_INVALID_ARG, "the autotuner tunes the FP32 regulariser");
    const SliceDesc &d0 = E->sl[0];
    hipStream_t st = E->stream;
    // synthetic test images on the first slice's layout
    std::vector<float> h((size_t)d0.N * d0.L * d0.L);
    unsigned x = 12345u;
    for (size_t k = 0; k < h.size(); ++k) {
        x = x * 1664525u + 1013904223u;
        h[k] = 0.01f + 0.01f * (float)((x >> 8) & 0xffff) / 65536.0f;
    }
    float *g = nullptr, *o4 = nullptr, *o8 = nullptr;
    SliceDesc *dd = nullptr;
    int *pre = nullptr, *xbd = nullptr;
    HIP_TRY(hipMalloc(&g, h.size() * sizeof(float)));
    HIP_TRY(hipMalloc(&o4, h.size() * sizeof(float)));
    HIP_TRY(hipMalloc(&o8, h.size() * sizeof(float)));
    HIP_TRY(hipMalloc(&dd, 2 * sizeof(SliceDesc)));
    HIP_TRY(hipMalloc(&pre, 4 * sizeof(int)));
    HIP_TRY(hipMalloc(&xbd, 18 * sizeof(int)));
    HIP_TRY(hipMemcpy(g, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    float ms[2] = {0, 0};
    const int cand[2] = {8, 4};
    std::vector<float> out[2];
    for (int c = 0; c < 2; ++c) {
        SliceDesc d = d0;
        d.img0 = 0;
        d.rp0 = 0;
        d.nrb = reg_blocks(d, E->prm.patch, cand[c]);
        const int hp[2] = {0, d.nrb};
        HIP_TRY(hipMemcpy(dd + c, &d, sizeof(SliceDesc), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(pre + 2 * c, hp, sizeof(hp), hipMemcpyHostToDevice));
        Batch bt = E->batch;
        bt.ns = 1;
        bt.sl = dd + c;
        bt.skip = nullptr;
        int xb[9];
        for (int x = 0; x <= 8; ++x) xb[x] = (int)((long long)d.nrb * x / 8);
        HIP_TRY(hipMemcpy(xbd + 9 * c, xb, sizeof(xb), hipMemcpyHostToDevice));
        Stage sg{pre + 2 * c, xbd + 9 * c, d.nrb, std::max(1, std::min(d.nrb, kCUs * 4)), 0};
        if (sg.grid >= 8) sg.grid -= sg.grid % 8;
        float *o = c == 0 ? o8 : o4;
        hipEvent_t a, b;
        HIP_TRY(hipEventCreate(&a));
        HIP_TRY(hipEventCreate(&b));
        launch_regularize(bt, sg, E->rp, cand[c], g, g, g, o, 1, nullptr, nullptr, st);   // warm-up
        HIP_TRY(hipEventRecord(a, st));
        for (int r = 0; r < 5; ++r) launch_regularize(bt, sg, E->rp, cand[c], g, g, g, o, 1, nullptr, nullptr, st);
        HIP_TRY(hipEventRecord(b, st));
        HIP_TRY(hipEventSynchronize(b));
        HIP_TRY(hipEventElapsedTime(&ms[c], a, b));
        ms[c] /= 5.0f;
        out[c].resize(h.size());
        HIP_TRY(hipMemcpy(out[c].data(), o, h.size() * sizeof(float), hipMemcpyDeviceToHost));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    (void)hipFree(g);
    (void)hipFree(o4);
    (void)hipFree(o8);
    (void)hipFree(dd);
    (void)hipFree(pre);
    (void)hipFree(xbd);
    const bool same = std::memcmp(out[0].data(), out[1].data(), out[0].size() * sizeof(float)) == 0;
    const int pick = (same && ms[1] < ms[0]) ? 4 : 8;
    if (chosen) *chosen = pick;
    if (ms_out) {
        ms_out[0] = ms[0];
        ms_out[1] = ms[1];
    }
    const std::string path = tune_cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {   // the cache is best effort: errors leave it unwritten
        std::error_code ec;
        std::filesystem::create_directories(path.substr(0, slash), ec);
    }
    std::ofstream fo(path, std::ios::app);
    if (fo)
        fo << "{\"key\": \"" << tune_key(E->prm, d0.L) << "\", \"rows_per_lane\": " << pick << ", \"ms8\": " << ms[0]
           << ", \"ms4\": " << ms[1] << ", \"bitwise_equal\": " << (same ? "true" : "false") << "}\n";
    if (!same) return fail(TNLM_E_HIP, "autotune candidates disagree bitwise; kept the reference tile");
    if (pick == E->rows_per_lane) return TNLM_OK;
    E->rows_per_lane = pick;
    // the regulariser's per-slice block counts depend on the tile height
    int rpp = 0;
    std::vector<int> creg;
    for (auto &d : E->sl) {
        d.nrb = reg_blocks(d, E->prm.patch, pick);
        d.rp0 = rpp;
        rpp += d.nrb;
        creg.push_back(d.nrb);
    }
    HIP_TRY(hipMemcpy(E->d_sl, E->sl.data(), E->sl.size() * sizeof(SliceDesc), hipMemcpyHostToDevice));
    HIP_TRY(E->alloc(&E->relpart, 2 * (size_t)rpp));
    tnlm_status s2 = make_stage(*E, E->st_reg, creg, kCUs * 4);
    E->drop_graph();
    return s2;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
#define CHECK_CTX()                                                                    \
    do {                                                                               \
        if (!ctx) return fail(TNLM_E_INVALID_ARG, "null context");                     \
    } while (0)

extern "C" tnlm_status tnlm_recon_init(tnlm_ctx **out, const tnlm_geometry *geom, const tnlm_params *params,
                                       void *stream) {
    if (!out) return fail(TNLM_E_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (!geom) return fail(TNLM_E_INVALID_ARG, "null geometry");
    std::unique_ptr<tnlm_ctx> c(new (std::nothrow) tnlm_ctx());
    if (!c) return fail(TNLM_E_OOM, "host allocation failed");
    tnlm_status s = engine_init(c->e, 1, geom, params, stream);
    if (s != TNLM_OK) return s;
    *out = c.release();
    return TNLM_OK;
}

extern "C" void tnlm_destroy(tnlm_ctx *ctx) { delete ctx; }

extern "C" tnlm_status tnlm_step(tnlm_ctx *ctx, const float *d_y, const float *d_w, float *d_f) {
    CHECK_CTX();
    if (!d_y || !d_w || !d_f) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    Engine *E = &ctx->e;
    E->cur = E->stream;
    if (E->prm.m1_cgls > 0) TIMED(E, K_VECTOR, launch_sqrt(d_w, E->cb.sw, E->nsino, E->stream));
    enqueue_step(E, E->batch, d_y, d_w, d_f);
    return last_launch();
}

extern "C" tnlm_status tnlm_solve(tnlm_ctx *ctx, const float *d_y, const float *d_w, float *d_f, int32_t *out_iters,
                                  float *out_rel) {
    CHECK_CTX();
    if (!d_y || !d_w || !d_f) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    tnlm_status s = engine_solve(&ctx->e, d_y, d_w, d_f);
    if (s != TNLM_OK) return s;
    tnlm_status ss = TNLM_OK;
    s = engine_results(&ctx->e, out_iters, out_rel, &ss);
    if (s == TNLM_E_NONFINITE) return fail(s, "an iterate became non-finite");
    if (s < 0) return s;
    if (s == TNLM_W_NOT_CONVERGED) g_last_error = "max_outer reached before tol_rel_update";
    return s;
}

extern "C" tnlm_status tnlm_get_history(tnlm_ctx *ctx, float *out, int32_t n, int32_t *out_n) {
    CHECK_CTX();
    Engine *E = &ctx->e;
    int cnt = 0;
    HIP_TRY(hipStreamSynchronize(E->stream));
    HIP_TRY(hipMemcpy(&cnt, E->counter(), sizeof(int), hipMemcpyDeviceToHost));
    cnt = std::min(cnt, E->prm.max_outer);
    if (out && n > 0) HIP_TRY(hipMemcpy(out, E->hist, sizeof(float) * std::min(n, cnt), hipMemcpyDeviceToHost));
    if (out_n) *out_n = cnt;
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_project(tnlm_ctx *ctx, const float *d_f, float *d_q) {
    CHECK_CTX();
    if (!d_f || !d_q) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    Engine *E = &ctx->e;
    E->cur = E->stream;
    TIMED(E, K_VECTOR, launch_transpose(E->batch, E->st_tr, d_f, E->fP, E->fTP, E->stream));
    TIMED(E, K_PROJECT, launch_project(E->batch, E->st_fp, PROJ_PLAIN, E->fP, E->fTP, nullptr, nullptr, d_q, nullptr,
                                       nullptr, E->stream));
    return last_launch();
}

extern "C" tnlm_status tnlm_backproject(tnlm_ctx *ctx, const float *d_q, float *d_f) {
    CHECK_CTX();
    if (!d_f || !d_q) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    Engine *E = &ctx->e;
    E->cur = E->stream;
    TIMED(E, K_BACKPROJECT, launch_backproject(E->batch, E->st_bp, d_q, d_f, nullptr, E->stream));
    return last_launch();
}

extern "C" tnlm_status tnlm_fbp(tnlm_ctx *ctx, const float *d_y, float *d_f, int32_t all_phases) {
    CHECK_CTX();
    if (!d_y || !d_f) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    Engine *E = &ctx->e;
    E->cur = E->stream;
    TIMED(E, K_FBP,
          launch_fbp(E->batch, E->st_ffilt, all_phases ? E->st_fbp_all : E->st_fbp_ph, d_y, E->hfilt, E->cw, E->Q, d_f,
                     all_phases ? 1 : 0, E->stream));
    return last_launch();
}

extern "C" tnlm_status tnlm_data_step(tnlm_ctx *ctx, const float *d_y, const float *d_w, const float *d_f,
                                      float *d_g) {
    CHECK_CTX();
    if (!d_y || !d_w || !d_f || !d_g) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    if (d_f == d_g) return fail(TNLM_E_INVALID_ARG, "d_f and d_g must not alias");
    Engine *E = &ctx->e;
    E->cur = E->stream;
    if (E->prm.m1_cgls > 0) TIMED(E, K_VECTOR, launch_sqrt(d_w, E->cb.sw, E->nsino, E->stream));
    enqueue_data_step(E, E->batch, d_y, d_w, d_f);
    TIMED(E, K_VECTOR, launch_copy(E->cb.u, d_g, E->nimg, E->stream));
    return last_launch();
}

extern "C" tnlm_status tnlm_regularize(tnlm_ctx *ctx, const float *d_guide, const float *d_value, const float *d_g,
                                       float *d_out, int32_t clamp) {
    CHECK_CTX();
    if (!d_guide || !d_value || !d_g || !d_out) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    if (d_out == d_guide || d_out == d_value || d_out == d_g)
        return fail(TNLM_E_INVALID_ARG, "d_out must not alias an input");
    Engine *E = &ctx->e;
    E->cur = E->stream;
    if (E->prm.ssd_mode == TNLM_SSD_BF16_MFMA)
        TIMED(E, K_REGULARIZE,
              launch_regularize_mfma(E->batch, E->st_reg, E->rp, d_guide, d_value, d_g, d_out, clamp ? 1 : 0, nullptr,
                                     nullptr, E->stream));
    else if (E->prm.ssd_mode == TNLM_SSD_FP32_SYMMETRIC)
        TIMED(E, K_REGULARIZE,
              launch_regularize_sym(E->batch, E->st_reg, E->rp, d_guide, d_value, d_g, d_out, clamp ? 1 : 0, nullptr,
                                    nullptr, E->symfwd, E->sympart, E->nimg, E->stream));
    else
        TIMED(E, K_REGULARIZE,
              launch_regularize(E->batch, E->st_reg, E->rp, E->rows_per_lane, d_guide, d_value, d_g, d_out,
                                clamp ? 1 : 0, nullptr, nullptr, E->stream));
    return last_launch();
}

extern "C" tnlm_status tnlm_data_cost(tnlm_ctx *ctx, const float *d_y, const float *d_w, const float *d_f,
                                      double *out) {
    CHECK_CTX();
    if (!d_y || !d_w || !d_f || !out) return fail(TNLM_E_INVALID_ARG, "null pointer");
    Engine *E = &ctx->e;
    E->cur = E->stream;
    TIMED(E, K_VECTOR, launch_transpose(E->batch, E->st_tr, d_f, E->fP, E->fTP, E->stream));
    TIMED(E, K_PROJECT, launch_project(E->batch, E->st_fp, PROJ_PLAIN, E->fP, E->fTP, nullptr, nullptr, E->cb.q,
                                       nullptr, nullptr, E->stream));
    const int nb = launch_wsq_sum(E->cb.q, d_y, d_w, E->nsino, E->cost_part, E->stream);
    std::vector<double> part(nb);
    HIP_TRY(hipMemcpyAsync(part.data(), E->cost_part, nb * sizeof(double), hipMemcpyDeviceToHost, E->stream));
    HIP_TRY(hipStreamSynchronize(E->stream));
    double s = 0.0;
    for (double v : part) s += v;
    *out = s;
    return last_launch();
}

extern "C" tnlm_status tnlm_cost(tnlm_ctx *ctx, const float *d_y, const float *d_w, const float *d_f,
                                 const float *d_guide, double *out_data, double *out_reg) {
    CHECK_CTX();
    if (!d_y || !d_w || !d_f || !d_guide || !out_data || !out_reg) return fail(TNLM_E_INVALID_ARG, "null pointer");
    tnlm_status s = tnlm_data_cost(ctx, d_y, d_w, d_f, out_data);
    if (s != TNLM_OK) return s;
    Engine *E = &ctx->e;
    const SliceDesc &d = E->sl[0];
    const int nb = launch_reg_cost(d.N, d.L, E->prm.patch, E->prm.window, E->prm.h, d_guide, d_f, E->cost_part, 1024,
                                   E->stream);
    std::vector<double> part(nb);
    HIP_TRY(hipMemcpyAsync(part.data(), E->cost_part, nb * sizeof(double), hipMemcpyDeviceToHost, E->stream));
    HIP_TRY(hipStreamSynchronize(E->stream));
    double r = 0.0;
    for (double v : part) r += v;
    *out_reg = r;
    return last_launch();
}

extern "C" tnlm_status tnlm_set_guide(tnlm_ctx *ctx, const float *d_guide) {
    CHECK_CTX();
    Engine *E = &ctx->e;
    HIP_TRY(hipStreamSynchronize(E->stream));
    if (E->fixed_guide != d_guide) E->drop_graph();   // the captured iteration reads the guide pointer
    E->fixed_guide = d_guide;
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_rel_change(tnlm_ctx *ctx, const float *d_a, const float *d_b, double *out) {
    CHECK_CTX();
    if (!d_a || !d_b || !out) return fail(TNLM_E_INVALID_ARG, "null pointer");
    Engine *E = &ctx->e;
    int *bad = E->nonfinite() + E->ns;   // spare flag slot
    launch_fill_int(bad, 1, 0, E->stream);
    const int nb = launch_diff_sq(d_a, d_b, E->nimg, E->cost_part, bad, E->stream);
    std::vector<double> part(2 * nb);
    int hb = 0;
    HIP_TRY(hipMemcpyAsync(part.data(), E->cost_part, part.size() * sizeof(double), hipMemcpyDeviceToHost, E->stream));
    HIP_TRY(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, E->stream));
    HIP_TRY(hipStreamSynchronize(E->stream));
    tnlm_status ls = last_launch();
    if (ls != TNLM_OK) return ls;
    if (hb) return fail(TNLM_E_NONFINITE, "non-finite value in an image stack");
    double d2 = 0.0, a2 = 0.0;
    for (int k = 0; k < nb; ++k) {
        d2 += part[2 * k];
        a2 += part[2 * k + 1];
    }
    *out = std::sqrt(d2) / std::max(std::sqrt(a2), 1e-30);
    return TNLM_OK;
}

static tnlm_status timing_enable(Engine *E, int32_t enable) {
    HIP_TRY(hipStreamSynchronize(E->stream));
    for (auto &r : E->recs) {
        E->pool.push_back(r.a);
        E->pool.push_back(r.b);
    }
    E->recs.clear();
    E->timing = enable != 0;
    return TNLM_OK;
}

static tnlm_status timing_read(Engine *E, double *ms, int32_t *launches) {
    if (!ms || !launches) return fail(TNLM_E_INVALID_ARG, "null output array");
    HIP_TRY(hipStreamSynchronize(E->stream));
    for (int k = 0; k < TNLM_KIND_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &r : E->recs) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.kind] += t;
        launches[r.kind] += 1;
        E->pool.push_back(r.a);
        E->pool.push_back(r.b);
    }
    E->recs.clear();
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_timing_enable(tnlm_ctx *ctx, int32_t enable) {
    CHECK_CTX();
    return timing_enable(&ctx->e, enable);
}

extern "C" tnlm_status tnlm_timing_read(tnlm_ctx *ctx, double *ms, int32_t *launches) {
    CHECK_CTX();
    return timing_read(&ctx->e, ms, launches);
}

extern "C" tnlm_status tnlm_autotune(tnlm_ctx *ctx, int32_t *rows_per_lane, float *ms) {
    CHECK_CTX();
    return engine_autotune(&ctx->e, rows_per_lane, ms);
}

// ---- batch of slices (ragged sizes)
extern "C" tnlm_status tnlm_batch_init(tnlm_batch **out, int32_t n_slices, const tnlm_geometry *geoms,
                                       const tnlm_params *params, void *stream) {
    if (!out) return fail(TNLM_E_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (n_slices < 1 || !geoms) return fail(TNLM_E_INVALID_ARG, "need n_slices >= 1 and geometries");
    std::unique_ptr<tnlm_batch> b(new (std::nothrow) tnlm_batch());
    if (!b) return fail(TNLM_E_OOM, "host allocation failed");
    tnlm_status s = engine_init(b->e, n_slices, geoms, params, stream);
    if (s != TNLM_OK) return s;
    Engine &E = b->e;
    HIP_TRY(E.alloc(&E.Y, E.nsino));
    HIP_TRY(E.alloc(&E.Wt, E.nsino));
    HIP_TRY(E.alloc(&E.F, E.nimg));
    *out = b.release();
    return TNLM_OK;
}

extern "C" void tnlm_batch_destroy(tnlm_batch *b) { delete b; }

static tnlm_status batch_solve(tnlm_batch *bt, const float *const *d_y, const float *const *d_w, float *const *d_f,
                               const int32_t *active, int32_t *out_iters, float *out_rel, tnlm_status *out_status) {
    if (!bt) return fail(TNLM_E_INVALID_ARG, "null batch");
    if (!d_y || !d_w || !d_f) return fail(TNLM_E_INVALID_ARG, "null pointer array");
    Engine *E = &bt->e;
    std::vector<char> act(E->ns, 1);
    if (active)
        for (int s = 0; s < E->ns; ++s) act[s] = active[s] != 0;
    for (int s = 0; s < E->ns; ++s)
        if (act[s] && (!d_y[s] || !d_w[s] || !d_f[s]))
            return fail(TNLM_E_INVALID_ARG, "null device pointer for slice " + std::to_string(s));
    hipStream_t st = E->stream;
    for (int s = 0; s < E->ns; ++s) {
        if (!act[s]) continue;
        const SliceDesc &d = E->sl[s];
        const size_t nsn = (size_t)d.N * d.V * d.B, ni = (size_t)d.N * d.L * d.L;
        HIP_TRY(hipMemcpyAsync(E->Y + d.sino0, d_y[s], nsn * sizeof(float), hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(E->Wt + d.sino0, d_w[s], nsn * sizeof(float), hipMemcpyDeviceToDevice, st));
        if (E->prm.init == TNLM_INIT_USER)
            HIP_TRY(hipMemcpyAsync(E->F + d.img0, d_f[s], ni * sizeof(float), hipMemcpyDeviceToDevice, st));
    }
    tnlm_status s = engine_solve(E, E->Y, E->Wt, E->F, active ? &act : nullptr);
    if (s != TNLM_OK) return s;
    for (int k = 0; k < E->ns; ++k) {
        if (!act[k]) continue;
        const SliceDesc &d = E->sl[k];
        HIP_TRY(hipMemcpyAsync(d_f[k], E->F + d.img0, (size_t)d.N * d.L * d.L * sizeof(float), hipMemcpyDeviceToDevice,
                               st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    s = engine_results(E, out_iters, out_rel, out_status);
    if (s < 0) return fail(s, "a slice failed (see out_status)");
    return s;
}

extern "C" tnlm_status tnlm_batch_solve(tnlm_batch *bt, const float *const *d_y, const float *const *d_w,
                                        float *const *d_f, int32_t *out_iters, float *out_rel,
                                        tnlm_status *out_status) {
    return batch_solve(bt, d_y, d_w, d_f, nullptr, out_iters, out_rel, out_status);
}

extern "C" tnlm_status tnlm_batch_solve_active(tnlm_batch *bt, const float *const *d_y, const float *const *d_w,
                                               float *const *d_f, const int32_t *active, int32_t *out_iters,
                                               float *out_rel, tnlm_status *out_status) {
    if (!active) return fail(TNLM_E_INVALID_ARG, "null active mask");
    return batch_solve(bt, d_y, d_w, d_f, active, out_iters, out_rel, out_status);
}

extern "C" tnlm_status tnlm_batch_timing_enable(tnlm_batch *b, int32_t enable) {
    if (!b) return fail(TNLM_E_INVALID_ARG, "null batch");
    return timing_enable(&b->e, enable);
}

extern "C" tnlm_status tnlm_batch_timing_read(tnlm_batch *b, double *ms, int32_t *launches) {
    if (!b) return fail(TNLM_E_INVALID_ARG, "null batch");
    return timing_read(&b->e, ms, launches);
}

// ---------------------------------------------------------------------------
// Regulariser sweep of one slice without a context and without allocation.
// The kernel's tables (slice descriptor, work-item prefix, XCD ranges) live in
// a library-owned device array; its address on each GPU is looked up once,
// with that GPU current, on the first call there.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = 1024;
constexpr size_t kScratchPre = 256, kScratchXb = 512;   // byte offsets of the prefix and XCD tables
static_assert(sizeof(SliceDesc) <= kScratchPre && kScratchPre + 2 * sizeof(int) <= kScratchXb &&
                  kScratchXb + 9 * sizeof(int) <= kNoAllocScratchBytes,
              "the tables of one slice fit the scratch array");
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

struct NoAllocTables {
    SliceDesc d;
    int pre[2];
    int xb[9];
};

// One lane writes the tables; the regulariser launched after it on the same
// stream reads them.
__global__ void k_write_noalloc_tables(unsigned char *dst, NoAllocTables t) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    *reinterpret_cast<SliceDesc *>(dst) = t.d;
    int *pre = reinterpret_cast<int *>(dst + kScratchPre);
    pre[0] = t.pre[0];
    pre[1] = t.pre[1];
    int *xb = reinterpret_cast<int *>(dst + kScratchXb);
    for (int k = 0; k < 9; ++k) xb[k] = t.xb[k];
}

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {};

static tnlm_status scratch_of_current_device(unsigned char **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(TNLM_E_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(TNLM_E_HIP, std::string("scratch address: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    return TNLM_OK;
}

extern "C" tnlm_status tnlm_regularize_noalloc(int32_t n_phases, int32_t L, int32_t patch, int32_t window, float h,
                                               float mu_hat, const float *d_guide, const float *d_value,
                                               const float *d_g, float *d_out, int32_t clamp, void *stream) {
    if (!d_guide || !d_value || !d_g || !d_out) return fail(TNLM_E_INVALID_ARG, "null device pointer");
    if (d_out == d_guide || d_out == d_value || d_out == d_g)
        return fail(TNLM_E_INVALID_ARG, "d_out must not alias an input");
    if (n_phases < 1 || L < 1 || L > 4096 || (long long)n_phases * L * L > (1LL << 31))
        return fail(TNLM_E_SHAPE, "need N >= 1, 1 <= L <= 4096 and N L^2 <= 2^31");
    if (!reg_supported(patch, window)) return fail(TNLM_E_INVALID_ARG, "patch must be odd in [3,9], window odd in [3,21]");
    if (window > L) return fail(TNLM_E_SHAPE, "window larger than the image");
    if (!(h > 0.0f) || !std::isfinite(h)) return fail(TNLM_E_INVALID_ARG, "h must be > 0");
    if (!(mu_hat >= 0.0f) || !std::isfinite(mu_hat)) return fail(TNLM_E_INVALID_ARG, "mu_hat must be >= 0");
    constexpr int kRowsPerLane = 4;   // any tile height gives the same bits
    NoAllocTables t{};
    t.d.N = n_phases;
    t.d.L = L;
    const long long items = (long long)reg_blocks(t.d, patch, kRowsPerLane);
    if (items < 1 || items > (1LL << 30)) return fail(TNLM_E_SHAPE, "too many regulariser tiles");
    t.d.nrb = (int)items;
    t.pre[0] = 0;
    t.pre[1] = (int)items;
    for (int x = 0; x <= 8; ++x) t.xb[x] = (int)(items * x / 8);
    unsigned char *ptr = nullptr;
    const tnlm_status ss = scratch_of_current_device(&ptr);
    if (ss != TNLM_OK) return ss;
    hipStream_t st = static_cast<hipStream_t>(stream);
    k_write_noalloc_tables<<<1, 64, 0, st>>>(ptr, t);
    Batch bt;
    bt.ns = 1;
    bt.sl = reinterpret_cast<const SliceDesc *>(ptr);
    Stage sg{reinterpret_cast<const int *>(ptr + kScratchPre), reinterpret_cast<const int *>(ptr + kScratchXb),
             (int)items, std::max(1, std::min((int)items, kCUs * 4)), 0};
    if (sg.grid >= 8) sg.grid -= sg.grid % 8;
    RegParams rp{patch, window, h, mu_hat};
    launch_regularize(bt, sg, rp, kRowsPerLane, d_guide, d_value, d_g, d_out, clamp ? 1 : 0, nullptr, nullptr, st);
    return last_launch();
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
