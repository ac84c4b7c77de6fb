// Launch descriptors shared by the network kernels (cnn.hip) and the host-side
// network (cnn_net.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace tnlm {

typedef unsigned short bf16b;   // raw BF16 bits

struct ConvFwd {
    const bf16b *in;
    int in_c0, in_ct;          // channel offset and channel count of the input tensor
    const bf16b *mask;         // optional: input multiplied by (mask > 0)
    int mask_c0, mask_ct;
    const bf16b *w;            // [Cout][Cin][ks][ks]
    const float *bias;         // [Cout] or null
    bf16b *out;                // optional BF16 output slice
    int out_c0, out_ct;
    float *out_f;              // optional FP32 output [n][Cout][H][W]
    const float *resid;        // optional FP32 residual added to out_f (same layout)
    float resid_scale;
    int n, Cin, Cout, H, W, ks, relu;
};

struct ConvWgrad {
    const bf16b *g;            // output gradient [n][g_ct][H][W], channels g_c0..
    int g_c0, g_ct;
    const bf16b *mask;         // layer output (ReLU mask) or null
    int mask_c0, mask_ct;
    const bf16b *in;           // layer input
    int in_c0, in_ct;
    float *partial;            // [nsplit][Cout][K]
    int n, Cin, Cout, H, W, ks, nsplit;
};

void cnn_conv_fwd(const ConvFwd &a, hipStream_t st);
void cnn_conv_wgrad(const ConvWgrad &a, hipStream_t st);
void cnn_wgrad_reduce(const float *partial, int nsplit, size_t n, float *gw, hipStream_t st);
// bias gradient; part: device scratch of Cout * n * cnn_bias_splits(n, HW, Cout) doubles
int cnn_bias_splits(int n, int HW, int Cout);
void cnn_bias_grad(const bf16b *g, int g_c0, int g_ct, const bf16b *mask, int mask_c0, int mask_ct, int n, int HW,
                   int Cout, double *part, float *gb, hipStream_t st);
void cnn_flip(const bf16b *w, bf16b *wt, int Cout, int Cin, int ks, hipStream_t st);
void cnn_to_bf16(const float *x, float s, bf16b *y, size_t n, hipStream_t st);
void cnn_pool_fwd(const bf16b *src, int c0, int ct, bf16b *dst, int n, int C, int H, int W, hipStream_t st);
void cnn_pool_bwd_add(const bf16b *g, bf16b *dst, int c0, int ct, int n, int C, int H, int W, hipStream_t st);
void cnn_up_fwd(const bf16b *src, int sc0, int sct, bf16b *dst, int dc0, int dct, int n, int C, int H, int W,
                hipStream_t st);
void cnn_up_bwd(const bf16b *g, int gc0, int gct, bf16b *dst, int dc0, int dct, int n, int C, int H, int W,
                hipStream_t st);
int cnn_mse(const float *out, const float *t, size_t n, float tscale, float gscale, bf16b *g, double *partial,
            hipStream_t st);
void cnn_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2, float eps, float c1,
              float c2, float ginv, bf16b *wb, size_t nw, hipStream_t st);
void cnn_f32_to_bf16(const float *x, bf16b *y, size_t n, hipStream_t st);
void cnn_fill_f32(float *x, size_t n, float v, hipStream_t st);
void cnn_fill_bf16(bf16b *x, size_t n, hipStream_t st);
void cnn_scale_copy(const float *x, float s, float *y, size_t n, hipStream_t st);
void cnn_count_nonfinite(const float *x, size_t n, int *flag, hipStream_t st);
void cnn_box_down(const float *src, float *dst, size_t nc, int H, int W, int f, hipStream_t st);
void cnn_bilinear_up(const float *src, float *dst, size_t nc, int h, int w, int f, hipStream_t st);

}  // namespace tnlm
