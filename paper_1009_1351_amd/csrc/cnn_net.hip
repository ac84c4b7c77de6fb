// Host side of the learned warm start: a 4-level U-Net (channels b, 2b, 4b, 8b;
// two 3x3 convolutions + ReLU per level, 2x2 average pooling, nearest 2x
// upsampling, skip concatenation, a 1x1 head and a residual connection to
// the input), trained with MSE and Adam by the kernels of cnn.hip.
//
// Input: the N per-phase FBP images of a slice as N channels (scaled by
// input_scale so values are O(1)); output: N channels in the same units,
// out = head(features) + input_scale * input.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "cnn_internal.h"
#include "internal.h"


using namespace tnlm;

namespace {
thread_local std::string g_cnn_error;
tnlm_status cfail(tnlm_status s, const std::string &m) {
    g_cnn_error = m;
    return s;
}
#define CHIP(expr)                                                                                           \
    do {                                                                                                     \
        hipError_t e_ = (expr);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            return cfail(e_ == hipErrorOutOfMemory ? TNLM_E_OOM : TNLM_E_HIP, std::string(#expr) + ": " +     \
                                                                                   hipGetErrorString(e_));    \
    } while (0)
}  // namespace

struct CnnLayer {
    int Cin, Cout, ks, relu;
    size_t w_off, b_off;
};

// Tensor = (buffer, channel offset, total channels); spatial size implied by the level.
struct TRef {
    bf16b *p;
    int c0, ct;
};

struct tnlm_cnn {
    hipStream_t stream = nullptr;
    int P = 10, b = 32;
    float scale = 50.0f;
    std::vector<CnnLayer> L;
    size_t nparams = 0, nweights = 0;
    float *Pm = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
    bf16b *Wb = nullptr, *Wt = nullptr;
    float *part = nullptr;
    size_t part_cap = 0;
    double *lpart = nullptr;
    double *bpart = nullptr;   // bias-gradient partials
    size_t bpart_cap = 0;
    int *flag = nullptr;
    long long step = 0;
    // activations for the current (n, H, W)
    int an = 0, aH = 0, aW = 0;
    std::vector<void *> act_allocs;
    bf16b *X, *a1, *cat1, *p1, *a2, *cat2, *p2, *a3, *cat3, *p3, *a4, *b4, *d3a, *d3, *d2a, *d2, *d1a, *d1, *gout;
    bf16b *gd1, *gd1a, *gcat1, *gd2, *gd2a, *gcat2, *gd3, *gd3a, *gcat3, *gb4, *ga4, *gp3, *ga3, *gp2, *ga2, *gp1, *ga1;
    float *outf = nullptr;
    float *rs = nullptr;   // resampled input and output of tnlm_cnn_forward_resampled
    size_t rs_cap = 0;

    ~tnlm_cnn() {
        (void)hipStreamSynchronize(stream);
        free_acts();
        for (void *p : {(void *)Pm, (void *)G, (void *)M, (void *)V, (void *)Wb, (void *)Wt, (void *)part, (void *)lpart,
                        (void *)bpart, (void *)flag, (void *)rs})
            if (p) (void)hipFree(p);
    }
    void free_acts() {
        for (void *p : act_allocs) (void)hipFree(p);
        act_allocs.clear();
        an = aH = aW = 0;
    }
};

static void add_layer(tnlm_cnn &c, int Cin, int Cout, int ks, int relu) {
    CnnLayer l{Cin, Cout, ks, relu, c.nweights, 0};
    c.nweights += (size_t)Cin * Cout * ks * ks;
    c.L.push_back(l);
}

// deterministic Gaussian init (xorshift64* + Box-Muller), He scaling
static void init_params(tnlm_cnn &c, unsigned long long seed, std::vector<float> &h) {
    h.assign(c.nparams, 0.0f);
    unsigned long long s = seed * 0x9E3779B97F4A7C15ULL + 1;
    auto next = [&]() {
        s ^= s >> 12;
        s ^= s << 25;
        s ^= s >> 27;
        return (double)((s * 0x2545F4914F6CDD1DULL) >> 11) / 9007199254740992.0;
    };
    for (size_t li = 0; li < c.L.size(); ++li) {
        const CnnLayer &l = c.L[li];
        const size_t n = (size_t)l.Cin * l.Cout * l.ks * l.ks;
        // the head starts near zero so the initial network is the identity (residual)
        const double sd = li + 1 == c.L.size() ? 1e-3 : std::sqrt(2.0 / (l.Cin * l.ks * l.ks));
        for (size_t k = 0; k < n; ++k) {
            const double u1 = std::max(next(), 1e-300), u2 = next();
            h[l.w_off + k] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    }
}

static tnlm_status alloc_acts(tnlm_cnn &c, int n, int H, int W) {
    if (n == c.an && H == c.aH && W == c.aW) return TNLM_OK;
    c.free_acts();
    const int b = c.b, P = c.P;
    const size_t s0 = (size_t)H * W, s1 = s0 / 4, s2 = s0 / 16, s3 = s0 / 64;
    auto A = [&](bf16b **p, size_t elems) -> hipError_t {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(elems, 1) * sizeof(bf16b));
        if (e == hipSuccess) {
            c.act_allocs.push_back(q);
            *p = (bf16b *)q;
        }
        return e;
    };
    const size_t N = n;
    CHIP(A(&c.X, N * P * s0));
    CHIP(A(&c.a1, N * b * s0));
    CHIP(A(&c.cat1, N * 3 * b * s0));
    CHIP(A(&c.p1, N * b * s1));
    CHIP(A(&c.a2, N * 2 * b * s1));
    CHIP(A(&c.cat2, N * 6 * b * s1));
    CHIP(A(&c.p2, N * 2 * b * s2));
    CHIP(A(&c.a3, N * 4 * b * s2));
    CHIP(A(&c.cat3, N * 12 * b * s2));
    CHIP(A(&c.p3, N * 4 * b * s3));
    CHIP(A(&c.a4, N * 8 * b * s3));
    CHIP(A(&c.b4, N * 8 * b * s3));
    CHIP(A(&c.d3a, N * 4 * b * s2));
    CHIP(A(&c.d3, N * 4 * b * s2));
    CHIP(A(&c.d2a, N * 2 * b * s1));
    CHIP(A(&c.d2, N * 2 * b * s1));
    CHIP(A(&c.d1a, N * b * s0));
    CHIP(A(&c.d1, N * b * s0));
    CHIP(A(&c.gout, N * P * s0));
    CHIP(A(&c.gd1, N * b * s0));
    CHIP(A(&c.gd1a, N * b * s0));
    CHIP(A(&c.gcat1, N * 3 * b * s0));
    CHIP(A(&c.gd2, N * 2 * b * s1));
    CHIP(A(&c.gd2a, N * 2 * b * s1));
    CHIP(A(&c.gcat2, N * 6 * b * s1));
    CHIP(A(&c.gd3, N * 4 * b * s2));
    CHIP(A(&c.gd3a, N * 4 * b * s2));
    CHIP(A(&c.gcat3, N * 12 * b * s2));
    CHIP(A(&c.gb4, N * 8 * b * s3));
    CHIP(A(&c.ga4, N * 8 * b * s3));
    CHIP(A(&c.gp3, N * 4 * b * s3));
    CHIP(A(&c.ga3, N * 4 * b * s2));
    CHIP(A(&c.gp2, N * 2 * b * s2));
    CHIP(A(&c.ga2, N * 2 * b * s1));
    CHIP(A(&c.gp1, N * b * s1));
    CHIP(A(&c.ga1, N * b * s0));
    void *q = nullptr;
    CHIP(hipMalloc(&q, N * P * s0 * sizeof(float)));
    c.act_allocs.push_back(q);
    c.outf = (float *)q;
    c.an = n;
    c.aH = H;
    c.aW = W;
    return TNLM_OK;
}

static void conv(tnlm_cnn &c, int li, TRef in, TRef out, int n, int H, int W, float *outf = nullptr,
                 const float *resid = nullptr) {
    const CnnLayer &l = c.L[li];
    ConvFwd a{};
    a.in = in.p;
    a.in_c0 = in.c0;
    a.in_ct = in.ct;
    a.mask = nullptr;
    a.w = c.Wb + l.w_off;
    a.bias = c.Pm + l.b_off;
    a.out = out.p;
    a.out_c0 = out.c0;
    a.out_ct = out.ct;
    a.out_f = outf;
    a.resid = resid;
    a.resid_scale = c.scale;
    a.n = n;
    a.Cin = l.Cin;
    a.Cout = l.Cout;
    a.H = H;
    a.W = W;
    a.ks = l.ks;
    a.relu = l.relu;
    cnn_conv_fwd(a, c.stream);
}

// forward pass; the input xin is FP32 [n][P][H][W] in image units
static void forward(tnlm_cnn &c, const float *xin, int n, int H, int W) {
    const int b = c.b, P = c.P;
    hipStream_t st = c.stream;
    const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
    cnn_to_bf16(xin, c.scale, c.X, (size_t)n * P * H * W, st);
    conv(c, 0, {c.X, 0, P}, {c.a1, 0, b}, n, H, W);
    conv(c, 1, {c.a1, 0, b}, {c.cat1, 2 * b, 3 * b}, n, H, W);             // e1 -> cat1[2b, 3b)
    cnn_pool_fwd(c.cat1, 2 * b, 3 * b, c.p1, n, b, H, W, st);
    conv(c, 2, {c.p1, 0, b}, {c.a2, 0, 2 * b}, n, H1, W1);
    conv(c, 3, {c.a2, 0, 2 * b}, {c.cat2, 4 * b, 6 * b}, n, H1, W1);       // e2 -> cat2[4b, 6b)
    cnn_pool_fwd(c.cat2, 4 * b, 6 * b, c.p2, n, 2 * b, H1, W1, st);
    conv(c, 4, {c.p2, 0, 2 * b}, {c.a3, 0, 4 * b}, n, H2, W2);
    conv(c, 5, {c.a3, 0, 4 * b}, {c.cat3, 8 * b, 12 * b}, n, H2, W2);      // e3 -> cat3[8b, 12b)
    cnn_pool_fwd(c.cat3, 8 * b, 12 * b, c.p3, n, 4 * b, H2, W2, st);
    conv(c, 6, {c.p3, 0, 4 * b}, {c.a4, 0, 8 * b}, n, H3, W3);
    conv(c, 7, {c.a4, 0, 8 * b}, {c.b4, 0, 8 * b}, n, H3, W3);
    cnn_up_fwd(c.b4, 0, 8 * b, c.cat3, 0, 12 * b, n, 8 * b, H2, W2, st);  // u3 -> cat3[0, 8b)
    conv(c, 8, {c.cat3, 0, 12 * b}, {c.d3a, 0, 4 * b}, n, H2, W2);
    conv(c, 9, {c.d3a, 0, 4 * b}, {c.d3, 0, 4 * b}, n, H2, W2);
    cnn_up_fwd(c.d3, 0, 4 * b, c.cat2, 0, 6 * b, n, 4 * b, H1, W1, st);   // u2 -> cat2[0, 4b)
    conv(c, 10, {c.cat2, 0, 6 * b}, {c.d2a, 0, 2 * b}, n, H1, W1);
    conv(c, 11, {c.d2a, 0, 2 * b}, {c.d2, 0, 2 * b}, n, H1, W1);
    cnn_up_fwd(c.d2, 0, 2 * b, c.cat1, 0, 3 * b, n, 2 * b, H, W, st);     // u1 -> cat1[0, 2b)
    conv(c, 12, {c.cat1, 0, 3 * b}, {c.d1a, 0, b}, n, H, W);
    conv(c, 13, {c.d1a, 0, b}, {c.d1, 0, b}, n, H, W);
    conv(c, 14, {c.d1, 0, b}, {nullptr, 0, 0}, n, H, W, c.outf, xin);     // head + residual
}

static int nsplit_for(const CnnLayer &l, long long P) {
    const int K = l.Cin * l.ks * l.ks;
    const int tiles = ((K + 63) / 64) * ((l.Cout + 63) / 64);
    // about 8 blocks per CU (256 CUs), at least 8 pixel chunks of 32 per split
    int ns = std::max(1, 2048 / tiles);
    ns = (int)std::min<long long>(ns, std::max<long long>(1, P / 256));
    return std::min(ns, 256);
}

// one layer's backward: gW, gb into c.G; input gradient into gin (if gin.p)
static tnlm_status layer_bwd(tnlm_cnn &c, int li, TRef g, TRef mask, TRef in, TRef gin, int n, int H, int W) {
    const CnnLayer &l = c.L[li];
    hipStream_t st = c.stream;
    const long long P = (long long)n * H * W;
    const int K = l.Cin * l.ks * l.ks;
    const int ns = nsplit_for(l, P);
    const size_t need = (size_t)ns * l.Cout * K;
    if (need > c.part_cap) {
        if (c.part) CHIP(hipFree(c.part));
        c.part = nullptr;
        CHIP(hipMalloc(&c.part, need * sizeof(float)));
        c.part_cap = need;
    }
    ConvWgrad wa{};
    wa.g = g.p;
    wa.g_c0 = g.c0;
    wa.g_ct = g.ct;
    wa.mask = mask.p;
    wa.mask_c0 = mask.c0;
    wa.mask_ct = mask.ct;
    wa.in = in.p;
    wa.in_c0 = in.c0;
    wa.in_ct = in.ct;
    wa.partial = c.part;
    wa.n = n;
    wa.Cin = l.Cin;
    wa.Cout = l.Cout;
    wa.H = H;
    wa.W = W;
    wa.ks = l.ks;
    wa.nsplit = ns;
    cnn_conv_wgrad(wa, st);
    cnn_wgrad_reduce(c.part, ns, (size_t)l.Cout * K, c.G + l.w_off, st);
    const size_t bneed = (size_t)l.Cout * n * cnn_bias_splits(n, H * W, l.Cout);
    if (bneed > c.bpart_cap) {
        if (c.bpart) CHIP(hipFree(c.bpart));
        c.bpart = nullptr;
        CHIP(hipMalloc(&c.bpart, bneed * sizeof(double)));
        c.bpart_cap = bneed;
    }
    cnn_bias_grad(g.p, g.c0, g.ct, mask.p, mask.c0, mask.ct, n, H * W, l.Cout, c.bpart, c.G + l.b_off, st);
    if (gin.p) {
        cnn_flip(c.Wb + l.w_off, c.Wt, l.Cout, l.Cin, l.ks, st);
        ConvFwd a{};
        a.in = g.p;
        a.in_c0 = g.c0;
        a.in_ct = g.ct;
        a.mask = mask.p;
        a.mask_c0 = mask.c0;
        a.mask_ct = mask.ct;
        a.w = c.Wt;
        a.bias = nullptr;
        a.out = gin.p;
        a.out_c0 = gin.c0;
        a.out_ct = gin.ct;
        a.n = n;
        a.Cin = l.Cout;
        a.Cout = l.Cin;
        a.H = H;
        a.W = W;
        a.ks = l.ks;
        a.relu = 0;
        cnn_conv_fwd(a, st);
    }
    return TNLM_OK;
}

static tnlm_status backward(tnlm_cnn &c, int n, int H, int W) {
    const int b = c.b, P = c.P;
    hipStream_t st = c.stream;
    const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
    const TRef none{nullptr, 0, 0};
    tnlm_status s;
#define LB(...) \
    if ((s = layer_bwd(c, __VA_ARGS__)) != TNLM_OK) return s
    LB(14, {c.gout, 0, P}, none, {c.d1, 0, b}, {c.gd1, 0, b}, n, H, W);
    LB(13, {c.gd1, 0, b}, {c.d1, 0, b}, {c.d1a, 0, b}, {c.gd1a, 0, b}, n, H, W);
    LB(12, {c.gd1a, 0, b}, {c.d1a, 0, b}, {c.cat1, 0, 3 * b}, {c.gcat1, 0, 3 * b}, n, H, W);
    cnn_up_bwd(c.gcat1, 0, 3 * b, c.gd2, 0, 2 * b, n, 2 * b, H, W, st);
    LB(11, {c.gd2, 0, 2 * b}, {c.d2, 0, 2 * b}, {c.d2a, 0, 2 * b}, {c.gd2a, 0, 2 * b}, n, H1, W1);
    LB(10, {c.gd2a, 0, 2 * b}, {c.d2a, 0, 2 * b}, {c.cat2, 0, 6 * b}, {c.gcat2, 0, 6 * b}, n, H1, W1);
    cnn_up_bwd(c.gcat2, 0, 6 * b, c.gd3, 0, 4 * b, n, 4 * b, H1, W1, st);
    LB(9, {c.gd3, 0, 4 * b}, {c.d3, 0, 4 * b}, {c.d3a, 0, 4 * b}, {c.gd3a, 0, 4 * b}, n, H2, W2);
    LB(8, {c.gd3a, 0, 4 * b}, {c.d3a, 0, 4 * b}, {c.cat3, 0, 12 * b}, {c.gcat3, 0, 12 * b}, n, H2, W2);
    cnn_up_bwd(c.gcat3, 0, 12 * b, c.gb4, 0, 8 * b, n, 8 * b, H2, W2, st);
    LB(7, {c.gb4, 0, 8 * b}, {c.b4, 0, 8 * b}, {c.a4, 0, 8 * b}, {c.ga4, 0, 8 * b}, n, H3, W3);
    LB(6, {c.ga4, 0, 8 * b}, {c.a4, 0, 8 * b}, {c.p3, 0, 4 * b}, {c.gp3, 0, 4 * b}, n, H3, W3);
    cnn_pool_bwd_add(c.gp3, c.gcat3, 8 * b, 12 * b, n, 4 * b, H2, W2, st);
    LB(5, {c.gcat3, 8 * b, 12 * b}, {c.cat3, 8 * b, 12 * b}, {c.a3, 0, 4 * b}, {c.ga3, 0, 4 * b}, n, H2, W2);
    LB(4, {c.ga3, 0, 4 * b}, {c.a3, 0, 4 * b}, {c.p2, 0, 2 * b}, {c.gp2, 0, 2 * b}, n, H2, W2);
    cnn_pool_bwd_add(c.gp2, c.gcat2, 4 * b, 6 * b, n, 2 * b, H1, W1, st);
    LB(3, {c.gcat2, 4 * b, 6 * b}, {c.cat2, 4 * b, 6 * b}, {c.a2, 0, 2 * b}, {c.ga2, 0, 2 * b}, n, H1, W1);
    LB(2, {c.ga2, 0, 2 * b}, {c.a2, 0, 2 * b}, {c.p1, 0, b}, {c.gp1, 0, b}, n, H1, W1);
    cnn_pool_bwd_add(c.gp1, c.gcat1, 2 * b, 3 * b, n, b, H, W, st);
    LB(1, {c.gcat1, 2 * b, 3 * b}, {c.cat1, 2 * b, 3 * b}, {c.a1, 0, b}, {c.ga1, 0, b}, n, H, W);
    LB(0, {c.ga1, 0, b}, {c.a1, 0, b}, {c.X, 0, P}, none, n, H, W);
#undef LB
    return TNLM_OK;
}

static tnlm_status check_shape(tnlm_cnn *c, int n, int H, int W) {
    if (!c) return cfail(TNLM_E_INVALID_ARG, "null network");
    if (n < 1 || H < 8 || W < 8 || H % 8 || W % 8 || (long long)n * H * W > (1LL << 28))
        return cfail(TNLM_E_SHAPE, "need n >= 1 and H, W multiples of 8");
    return TNLM_OK;
}

static tnlm_status loss_and_grad(tnlm_cnn *c, const float *in, const float *tgt, int n, int H, int W, double *loss) {
    tnlm_status s = alloc_acts(*c, n, H, W);
    if (s != TNLM_OK) return s;
    forward(*c, in, n, H, W);
    const size_t cnt = (size_t)n * c->P * H * W;
    const int nb = cnn_mse(c->outf, tgt, cnt, c->scale, 1.0f, c->gout, c->lpart, c->stream);
    s = backward(*c, n, H, W);
    if (s != TNLM_OK) return s;
    std::vector<double> lp(nb);
    CHIP(hipMemcpyAsync(lp.data(), c->lpart, nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CHIP(hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (double v : lp) tot += v;
    if (loss) *loss = tot / (double)cnt;
    CHIP(hipGetLastError());
    return TNLM_OK;
}

extern "C" {

tnlm_status tnlm_cnn_create(tnlm_cnn **out, int32_t phases, int32_t base_channels, uint64_t seed, float input_scale,
                            void *stream) {
    if (!out) return cfail(TNLM_E_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (phases < 1 || phases > 64 || base_channels < 8 || base_channels > 128 || base_channels % 8 || !(input_scale > 0))
        return cfail(TNLM_E_INVALID_ARG, "need 1 <= phases <= 64, base channels a multiple of 8 in [8, 128], scale > 0");
    std::unique_ptr<tnlm_cnn> c(new (std::nothrow) tnlm_cnn());
    if (!c) return cfail(TNLM_E_OOM, "host allocation failed");
    c->stream = (hipStream_t)stream;
    c->P = phases;
    c->b = base_channels;
    c->scale = input_scale;
    const int b = base_channels, P = phases;
    add_layer(*c, P, b, 3, 1);
    add_layer(*c, b, b, 3, 1);
    add_layer(*c, b, 2 * b, 3, 1);
    add_layer(*c, 2 * b, 2 * b, 3, 1);
    add_layer(*c, 2 * b, 4 * b, 3, 1);
    add_layer(*c, 4 * b, 4 * b, 3, 1);
    add_layer(*c, 4 * b, 8 * b, 3, 1);
    add_layer(*c, 8 * b, 8 * b, 3, 1);
    add_layer(*c, 12 * b, 4 * b, 3, 1);
    add_layer(*c, 4 * b, 4 * b, 3, 1);
    add_layer(*c, 6 * b, 2 * b, 3, 1);
    add_layer(*c, 2 * b, 2 * b, 3, 1);
    add_layer(*c, 3 * b, b, 3, 1);
    add_layer(*c, b, b, 3, 1);
    add_layer(*c, b, P, 1, 0);
    size_t off = c->nweights;
    size_t maxw = 0;
    for (auto &l : c->L) {
        l.b_off = off;
        off += l.Cout;
        maxw = std::max(maxw, (size_t)l.Cin * l.Cout * l.ks * l.ks);
    }
    c->nparams = off;
    std::vector<float> h;
    init_params(*c, seed, h);
    CHIP(hipMalloc(&c->Pm, c->nparams * sizeof(float)));
    CHIP(hipMalloc(&c->G, c->nparams * sizeof(float)));
    CHIP(hipMalloc(&c->M, c->nparams * sizeof(float)));
    CHIP(hipMalloc(&c->V, c->nparams * sizeof(float)));
    CHIP(hipMalloc(&c->Wb, c->nweights * sizeof(bf16b)));
    CHIP(hipMalloc(&c->Wt, maxw * sizeof(bf16b)));
    CHIP(hipMalloc(&c->lpart, 1024 * sizeof(double)));
    CHIP(hipMalloc(&c->flag, sizeof(int)));
    CHIP(hipMemcpy(c->Pm, h.data(), c->nparams * sizeof(float), hipMemcpyHostToDevice));
    cnn_fill_f32(c->M, c->nparams, 0.0f, c->stream);
    cnn_fill_f32(c->V, c->nparams, 0.0f, c->stream);
    cnn_fill_f32(c->G, c->nparams, 0.0f, c->stream);
    cnn_f32_to_bf16(c->Pm, c->Wb, c->nweights, c->stream);
    CHIP(hipStreamSynchronize(c->stream));
    CHIP(hipGetLastError());
    *out = c.release();
    return TNLM_OK;
}

void tnlm_cnn_destroy(tnlm_cnn *c) { delete c; }

int64_t tnlm_cnn_num_params(const tnlm_cnn *c) { return c ? (int64_t)c->nparams : -1; }

tnlm_status tnlm_cnn_get_params(tnlm_cnn *c, float *host, int64_t n) {
    if (!c || !host || n != (int64_t)c->nparams) return cfail(TNLM_E_INVALID_ARG, "need a buffer of num_params floats");
    CHIP(hipStreamSynchronize(c->stream));
    CHIP(hipMemcpy(host, c->Pm, c->nparams * sizeof(float), hipMemcpyDeviceToHost));
    return TNLM_OK;
}

tnlm_status tnlm_cnn_set_params(tnlm_cnn *c, const float *host, int64_t n) {
    if (!c || !host || n != (int64_t)c->nparams) return cfail(TNLM_E_INVALID_ARG, "need a buffer of num_params floats");
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(host[k])) return cfail(TNLM_E_NONFINITE, "non-finite parameter");
    CHIP(hipStreamSynchronize(c->stream));
    CHIP(hipMemcpy(c->Pm, host, c->nparams * sizeof(float), hipMemcpyHostToDevice));
    cnn_f32_to_bf16(c->Pm, c->Wb, c->nweights, c->stream);
    CHIP(hipStreamSynchronize(c->stream));
    return TNLM_OK;
}

tnlm_status tnlm_cnn_forward(tnlm_cnn *c, const float *d_in, float *d_out, int32_t n, int32_t H, int32_t W) {
    tnlm_status s = check_shape(c, n, H, W);
    if (s != TNLM_OK) return s;
    if (!d_in || !d_out) return cfail(TNLM_E_INVALID_ARG, "null device pointer");
    if ((s = alloc_acts(*c, n, H, W)) != TNLM_OK) return s;
    forward(*c, d_in, n, H, W);
    cnn_scale_copy(c->outf, 1.0f / c->scale, d_out, (size_t)n * c->P * H * W, c->stream);
    CHIP(hipGetLastError());
    return TNLM_OK;
}

tnlm_status tnlm_cnn_forward_resampled(tnlm_cnn *c, const float *d_in, float *d_out, int32_t n, int32_t H, int32_t W,
                                       int32_t factor) {
    if (factor == 1) return tnlm_cnn_forward(c, d_in, d_out, n, H, W);
    if (!c) return cfail(TNLM_E_INVALID_ARG, "null network");
    if (factor != 2 && factor != 4 && factor != 8) return cfail(TNLM_E_INVALID_ARG, "factor must be 1, 2, 4 or 8");
    if (n < 1 || H < 1 || W < 1 || H % factor || W % factor)
        return cfail(TNLM_E_SHAPE, "H and W must be positive multiples of the factor");
    if (!d_in || !d_out) return cfail(TNLM_E_INVALID_ARG, "null device pointer");
    const int h = H / factor, w = W / factor;
    tnlm_status s = check_shape(c, n, h, w);
    if (s != TNLM_OK) return s;
    const size_t ns = (size_t)n * c->P * h * w;
    if (c->rs_cap < 2 * ns) {
        CHIP(hipStreamSynchronize(c->stream));
        if (c->rs) (void)hipFree(c->rs);
        c->rs = nullptr;
        c->rs_cap = 0;
        CHIP(hipMalloc(&c->rs, 2 * ns * sizeof(float)));
        c->rs_cap = 2 * ns;
    }
    cnn_box_down(d_in, c->rs, (size_t)n * c->P, H, W, factor, c->stream);
    if ((s = tnlm_cnn_forward(c, c->rs, c->rs + ns, n, h, w)) != TNLM_OK) return s;
    cnn_bilinear_up(c->rs + ns, d_out, (size_t)n * c->P, h, w, factor, c->stream);
    CHIP(hipGetLastError());
    return TNLM_OK;
}

tnlm_status tnlm_image_upsample(const float *d_in, float *d_out, int32_t n, int32_t h, int32_t w, int32_t factor,
                                void *stream) {
    if (!d_in || !d_out) return cfail(TNLM_E_INVALID_ARG, "null device pointer");
    if (n < 1 || h < 1 || w < 1 || factor < 1 || factor > 16) return cfail(TNLM_E_SHAPE, "bad image count or size");
    if ((long long)n * h * w * factor * factor > (1LL << 31)) return cfail(TNLM_E_SHAPE, "output too large");
    cnn_bilinear_up(d_in, d_out, (size_t)n, h, w, factor, (hipStream_t)stream);
    CHIP(hipGetLastError());
    return TNLM_OK;
}

tnlm_status tnlm_cnn_loss_grad(tnlm_cnn *c, const float *d_in, const float *d_target, int32_t n, int32_t H, int32_t W,
                               double *loss, float *host_grad, int64_t ngrad) {
    tnlm_status s = check_shape(c, n, H, W);
    if (s != TNLM_OK) return s;
    if (!d_in || !d_target) return cfail(TNLM_E_INVALID_ARG, "null device pointer");
    if ((s = loss_and_grad(c, d_in, d_target, n, H, W, loss)) != TNLM_OK) return s;
    if (host_grad) {
        if (ngrad != (int64_t)c->nparams) return cfail(TNLM_E_INVALID_ARG, "gradient buffer must hold num_params floats");
        CHIP(hipMemcpy(host_grad, c->G, c->nparams * sizeof(float), hipMemcpyDeviceToHost));
    }
    return TNLM_OK;
}

tnlm_status tnlm_cnn_train_step(tnlm_cnn *c, const float *d_in, const float *d_target, int32_t n, int32_t H, int32_t W,
                                float lr, double *loss) {
    tnlm_status s = check_shape(c, n, H, W);
    if (s != TNLM_OK) return s;
    if (!d_in || !d_target || !(lr > 0)) return cfail(TNLM_E_INVALID_ARG, "null device pointer or lr <= 0");
    double l = 0.0;
    if ((s = loss_and_grad(c, d_in, d_target, n, H, W, &l)) != TNLM_OK) return s;
    if (!std::isfinite(l)) return cfail(TNLM_E_NONFINITE, "non-finite loss");
    c->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)c->step), c2 = 1.0f - std::pow(b2, (float)c->step);
    cnn_adam(c->Pm, c->G, c->M, c->V, c->nparams, lr, b1, b2, 1e-8f, c1, c2, 1.0f, c->Wb, c->nweights, c->stream);
    CHIP(hipGetLastError());
    if (loss) *loss = l;
    return TNLM_OK;
}

// checkpoint: magic, version, phases, base, scale, step, nparams, params, m, v
tnlm_status tnlm_cnn_save(tnlm_cnn *c, const char *path) {
    if (!c || !path) return cfail(TNLM_E_INVALID_ARG, "null argument");
    std::vector<float> p(c->nparams), m(c->nparams), v(c->nparams);
    CHIP(hipStreamSynchronize(c->stream));
    CHIP(hipMemcpy(p.data(), c->Pm, c->nparams * 4, hipMemcpyDeviceToHost));
    CHIP(hipMemcpy(m.data(), c->M, c->nparams * 4, hipMemcpyDeviceToHost));
    CHIP(hipMemcpy(v.data(), c->V, c->nparams * 4, hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return cfail(TNLM_E_INVALID_ARG, std::string("cannot write ") + path);
    const char magic[8] = {'T', 'N', 'L', 'M', 'C', 'N', 'N', '1'};
    const int32_t hdr[2] = {c->P, c->b};
    const int64_t hdr2[2] = {c->step, (int64_t)c->nparams};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 2, f) == 2 && std::fwrite(&c->scale, 4, 1, f) == 1 &&
              std::fwrite(hdr2, 8, 2, f) == 2 && std::fwrite(p.data(), 4, p.size(), f) == p.size() &&
              std::fwrite(m.data(), 4, m.size(), f) == m.size() && std::fwrite(v.data(), 4, v.size(), f) == v.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? TNLM_OK : cfail(TNLM_E_INVALID_ARG, "short write");
}

tnlm_status tnlm_cnn_load(tnlm_cnn *c, const char *path) {
    if (!c || !path) return cfail(TNLM_E_INVALID_ARG, "null argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return cfail(TNLM_E_INVALID_ARG, std::string("cannot read ") + path);
    char magic[8];
    int32_t hdr[2];
    float scale;
    int64_t hdr2[2];
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "TNLMCNN1", 8) == 0 && std::fread(hdr, 4, 2, f) == 2 &&
              std::fread(&scale, 4, 1, f) == 1 && std::fread(hdr2, 8, 2, f) == 2 && hdr[0] == c->P && hdr[1] == c->b &&
              hdr2[1] == (int64_t)c->nparams && hdr2[0] >= 0;
    std::vector<float> p(c->nparams), m(c->nparams), v(c->nparams);
    ok = ok && std::fread(p.data(), 4, p.size(), f) == p.size() && std::fread(m.data(), 4, m.size(), f) == m.size() &&
         std::fread(v.data(), 4, v.size(), f) == v.size();
    std::fclose(f);
    if (!ok) return cfail(TNLM_E_INVALID_ARG, "not a checkpoint of this network (magic, shape or length mismatch)");
    for (size_t k = 0; k < p.size(); ++k)
        if (!std::isfinite(p[k]) || !std::isfinite(m[k]) || !std::isfinite(v[k]) || v[k] < 0)
            return cfail(TNLM_E_NONFINITE, "checkpoint holds non-finite values");
    if (!(scale > 0) || !std::isfinite(scale)) return cfail(TNLM_E_INVALID_ARG, "bad input scale in checkpoint");
    CHIP(hipStreamSynchronize(c->stream));
    CHIP(hipMemcpy(c->Pm, p.data(), c->nparams * 4, hipMemcpyHostToDevice));
    CHIP(hipMemcpy(c->M, m.data(), c->nparams * 4, hipMemcpyHostToDevice));
    CHIP(hipMemcpy(c->V, v.data(), c->nparams * 4, hipMemcpyHostToDevice));
    c->scale = scale;
    c->step = hdr2[0];
    cnn_f32_to_bf16(c->Pm, c->Wb, c->nweights, c->stream);
    CHIP(hipStreamSynchronize(c->stream));
    return TNLM_OK;
}

const char *tnlm_cnn_last_error(void) { return g_cnn_error.c_str(); }

}  // extern "C"
