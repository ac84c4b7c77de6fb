// Kernels of the learned warm start: a U-Net style encoder-decoder mapping the
// N per-phase FBP images of a slice to an estimate of its TNLM solution, used
// as f^(0) of the TNLM algorithm box instead of the FBP of all phases.
//
// Tensors are NCHW. Activations and weights are BF16 (stored as raw 16-bit
// patterns), accumulation is FP32, master weights and Adam moments FP32.
// 3x3 and 1x1 convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16:
//   forward      out[co][p]  = sum_k W[co][k] col[k][p],     k = (ci, ky, kx)
//   input grad   = forward convolution of the masked output gradient with the
//                  flipped, transposed weights
//   weight grad  gW[co][k]   = sum_p g[co][p] col[k][p]   (split over pixel
//                  ranges, partials reduced in a fixed order: deterministic)
// A block computes a 64 x 64 output tile with 4 waves of 32 x 32 (2 x 2 MFMA
// tiles); K advances in chunks of 32 staged in LDS, both operands stored with
// the K index contiguous so every lane's 8 K-values are one 16-byte read.
#include "cnn_internal.h"
#include "devutil.h"
#include "internal.h"

namespace tnlm {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16b f2b(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }
__device__ __forceinline__ float b2f(bf16b b) { return __builtin_bit_cast(float, (unsigned)b << 16); }

constexpr int kT = 64;     // tile edge (rows of the output matrix and columns)
constexpr int kKC = 32;    // K chunk
constexpr int kLdsK = 40;  // padded K stride in LDS (elements): 80 bytes, 16-byte aligned rows

// ---------------------------------------------------------------------------
// forward convolution (also used for the input gradient)
// ---------------------------------------------------------------------------

// KS: the kernel size when known at compile time (1 or 3), 0 for any (a.ks).
// Each chunk's operands are loaded into registers one chunk ahead (issued
// before the current chunk's matrix operations), then stored to LDS.
template <int KS>
__global__ __launch_bounds__(kBlock) void k_conv_fwd(ConvFwd a) {
    static_assert(kT == 64 && kBlock == 4 * kT && kKC == 32, "one pixel and 8 K-values per thread in staging");
    static_assert(kT * kKC == 8 * kBlock, "8 weight values per thread in staging");
    __shared__ __attribute__((aligned(16))) bf16b sA[kT * kLdsK];
    __shared__ __attribute__((aligned(16))) bf16b sB[kT * kLdsK];
    const int ks = KS > 0 ? KS : a.ks, ks2 = ks * ks, pad = ks / 2;
    const int HW = a.H * a.W, K = a.Cin * ks2;
    const int p0 = blockIdx.x * kT, co0 = blockIdx.y * kT, nimg = blockIdx.z;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int l16 = lane & 15, kg = lane >> 4;
    f4_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = (f4_t){0.0f, 0.0f, 0.0f, 0.0f};
    const bf16b *inb = a.in + ((size_t)nimg * a.in_ct + a.in_c0) * HW;
    const bf16b *mb = a.mask ? a.mask + ((size_t)nimg * a.mask_ct + a.mask_c0) * HW : nullptr;
    // weight staging: element e = threadIdx.x + kBlock j of the chunk, row e / kKC, column e % kKC
    const int ar = threadIdx.x / kKC, ac = threadIdx.x % kKC;   // rows ar + (kBlock / kKC) j
    // im2col staging: pixel p0 + pr and K-values [8 kq, 8 kq + 8) of each chunk;
    // kq is the wave's index, so the K-values' (ci, ky, kx) are the same for
    // the whole wave (scalar registers) and a lane only tests its pixel's
    // neighbour mask (bit ky * ks + kx: neighbour inside the image)
    const int pr = threadIdx.x & (kT - 1), kq = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool pix = p0 + pr < HW;
    const int ypix = pix ? (p0 + pr) / a.W : 0, xpix = pix ? p0 + pr - ypix * a.W : 0;
    const int pixoff = ypix * a.W + xpix;
    unsigned nbr = 0;
    if (KS > 0 && pix) {
#pragma unroll
        for (int ky = 0; ky < KS; ++ky)
#pragma unroll
            for (int kx = 0; kx < KS; ++kx)
                if ((unsigned)(ypix + ky - pad) < (unsigned)a.H && (unsigned)(xpix + kx - pad) < (unsigned)a.W)
                    nbr |= 1u << (ky * KS + kx);
    }
    auto load_chunk = [&](int kc, u16x8 &av, u16x8 &bv) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {   // A: weights rows co0.., K columns kc..
            const int co = co0 + ar + (kBlock / kKC) * j, k = kc + ac;
            av[j] = (co < a.Cout && k < K) ? a.w[(size_t)co * K + k] : (bf16b)0;
        }
        // B: im2col, stored [pixel][k]; the thread's 8 K-values of its pixel
        // (consecutive lanes on consecutive pixels)
        int k = kc + 8 * kq;
        if constexpr (KS > 0) {
            int ci = k / (KS * KS), kk = k - ci * (KS * KS);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int ky = kk / KS, kx = kk - ky * KS;
                const bool ok = k < K && ((nbr >> kk) & 1u) != 0;
                // a lane without the value reads the tensor's first element instead
                const int off = ok ? ci * HW + pixoff + (ky - pad) * a.W + (kx - pad) : 0;
                bf16b v = inb[off];
                if (mb && !(b2f(mb[off]) > 0.0f)) v = 0;
                bv[t] = ok ? v : (bf16b)0;
                ++k;
                if (++kk == KS * KS) {
                    kk = 0;
                    ++ci;
                }
            }
        } else {
            int ci = k / ks2, kk = k - ci * ks2;
            int ky = kk / ks, kx = kk - ky * ks;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                bf16b v = 0;
                if (pix && k < K) {
                    const int y = ypix + ky - pad, x = xpix + kx - pad;
                    if ((unsigned)y < (unsigned)a.H && (unsigned)x < (unsigned)a.W) {
                        const size_t off = (size_t)ci * HW + (size_t)y * a.W + x;
                        v = inb[off];
                        if (mb && !(b2f(mb[off]) > 0.0f)) v = 0;
                    }
                }
                bv[t] = v;
                ++k;
                if (++kx == ks) {
                    kx = 0;
                    if (++ky == ks) {
                        ky = 0;
                        ++ci;
                    }
                }
            }
        }
    };
    u16x8 av, bv;
    load_chunk(0, av, bv);
    for (int kc = 0; kc < K; kc += kKC) {
#pragma unroll
        for (int j = 0; j < 8; ++j) sA[(ar + (kBlock / kKC) * j) * kLdsK + ac] = av[j];
        *(u16x8 *)(sB + pr * kLdsK + 8 * kq) = bv;
        __syncthreads();
        if (kc + kKC < K) load_chunk(kc + kKC, av, bv);   // in flight during this chunk's products
        bf16x8_t fa[2], fb[2];
        for (int i = 0; i < 2; ++i) {
            const u16x8 va = *(const u16x8 *)(sA + (wm * 32 + i * 16 + l16) * kLdsK + 8 * kg);
            fa[i] = __builtin_bit_cast(bf16x8_t, va);
            const u16x8 vb = *(const u16x8 *)(sB + (wn * 32 + i * 16 + l16) * kLdsK + 8 * kg);
            fb[i] = __builtin_bit_cast(bf16x8_t, vb);
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // epilogue: acc[i][j][t] = out[co = co0 + wm*32 + i*16 + 4kg + t][p = p0 + wn*32 + j*16 + l16]
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int t = 0; t < 4; ++t) {
                const int co = co0 + wm * 32 + i * 16 + 4 * kg + t, p = p0 + wn * 32 + j * 16 + l16;
                if (co >= a.Cout || p >= HW) continue;
                float v = acc[i][j][t] + (a.bias ? a.bias[co] : 0.0f);
                if (a.relu) v = fmaxf(v, 0.0f);
                if (a.out) a.out[((size_t)nimg * a.out_ct + a.out_c0 + co) * HW + p] = f2b(v);
                if (a.out_f) {
                    const size_t e = ((size_t)nimg * a.Cout + co) * HW + p;
                    a.out_f[e] = a.resid ? fmaf(a.resid_scale, a.resid[e], v) : v;
                }
            }
}

// ---------------------------------------------------------------------------
// weight gradient: partial[split][co][k] = sum over a pixel range of
// g[co][p] * (mask>0) * col[k][p]; all images of the batch are one pixel axis
// ---------------------------------------------------------------------------

template <int KS>
__global__ __launch_bounds__(kBlock) void k_conv_wgrad(ConvWgrad a) {
    static_assert(kBlock % kKC == 0 && kT % (kBlock / kKC) == 0, "whole rows per staging pass");
    __shared__ __attribute__((aligned(16))) bf16b sA[kT * kLdsK];   // [co][p]
    __shared__ __attribute__((aligned(16))) bf16b sB[kT * kLdsK];   // [k][p]
    const int ks = KS > 0 ? KS : a.ks, ks2 = ks * ks, pad = ks / 2;
    const int HW = a.H * a.W, K = a.Cin * ks2;
    const long long P = (long long)a.n * HW;
    const int k0 = blockIdx.x * kT, co0 = blockIdx.y * kT, split = blockIdx.z;
    const long long per = ((P + a.nsplit - 1) / a.nsplit + kKC - 1) / kKC * kKC;
    const long long pb = (long long)split * per, pe = std::min(P, pb + per);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int l16 = lane & 15, kg = lane >> 4;
    f4_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = (f4_t){0.0f, 0.0f, 0.0f, 0.0f};
    // staging: the thread's pixel column cB of each chunk, rows rB, rB + 8, ...
    // of both tiles; the pixel's image, row and column are found once and
    // advanced by kKC pixels per chunk
    const int cB = threadIdx.x % kKC, rB = threadIdx.x / kKC;
    int img = 0, yy = 0, xx = 0;
    if (pb + cB < P) {
        img = (int)((pb + cB) / HW);
        const int p = (int)(pb + cB - (long long)img * HW);
        yy = p / a.W;
        xx = p - yy * a.W;
    }
    // one chunk's operands into registers, then the pixel advanced by kKC
    auto load_chunk = [&](long long pc, u16x8 &av, u16x8 &bv) {
        const bool live = pc + cB < pe;
        const int p = yy * a.W + xx;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int co = co0 + rB + (kBlock / kKC) * j;
            bf16b v = 0;
            if (co < a.Cout && live) {
                v = a.g[((size_t)img * a.g_ct + a.g_c0 + co) * HW + p];
                if (a.mask && !(b2f(a.mask[((size_t)img * a.mask_ct + a.mask_c0 + co) * HW + p]) > 0.0f)) v = 0;
            }
            av[j] = v;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k0 + rB + (kBlock / kKC) * j;
            bf16b v = 0;
            if (k < K && live) {
                const int ci = k / ks2, kk = k - ci * ks2;   // divisions by constants when KS > 0
                const int ky = kk / ks, kx = kk - ky * ks;
                const int y = yy + ky - pad, x = xx + kx - pad;
                if ((unsigned)y < (unsigned)a.H && (unsigned)x < (unsigned)a.W)
                    v = a.in[((size_t)img * a.in_ct + a.in_c0 + ci) * HW + (size_t)y * a.W + x];
            }
            bv[j] = v;
        }
        xx += kKC;
        while (xx >= a.W) {
            xx -= a.W;
            if (++yy == a.H) {
                yy = 0;
                ++img;
            }
        }
    };
    static_assert(kT == 8 * (kBlock / kKC), "8 rows of each tile per thread");
    u16x8 av, bv;
    if (pb < pe) load_chunk(pb, av, bv);
    for (long long pc = pb; pc < pe; pc += kKC) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            sA[(rB + (kBlock / kKC) * j) * kLdsK + cB] = av[j];
            sB[(rB + (kBlock / kKC) * j) * kLdsK + cB] = bv[j];
        }
        __syncthreads();
        if (pc + kKC < pe) load_chunk(pc + kKC, av, bv);   // in flight during this chunk's products
        bf16x8_t fa[2], fb[2];
        for (int i = 0; i < 2; ++i) {
            fa[i] = __builtin_bit_cast(bf16x8_t, *(const u16x8 *)(sA + (wm * 32 + i * 16 + l16) * kLdsK + 8 * kg));
            fb[i] = __builtin_bit_cast(bf16x8_t, *(const u16x8 *)(sB + (wn * 32 + i * 16 + l16) * kLdsK + 8 * kg));
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int t = 0; t < 4; ++t) {
                const int co = co0 + wm * 32 + i * 16 + 4 * kg + t, k = k0 + wn * 32 + j * 16 + l16;
                if (co < a.Cout && k < K) a.partial[((size_t)split * a.Cout + co) * K + k] = acc[i][j][t];
            }
}

// gW = sum over splits in order; gb[co] = sum over pixels of the masked gradient
__global__ void k_wgrad_reduce(const float *__restrict__ partial, int nsplit, size_t n, float *__restrict__ gw) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int k = 0; k < nsplit; ++k) s += partial[(size_t)k * n + e];
        gw[e] = s;
    }
}

// bias gradient in two steps: part[co][img * nsp + sp] = sum over the pixel
// range sp of image img of the masked output gradient (one block each), then
// gb[co] = the sum of the co's partials in order (deterministic)
__global__ __launch_bounds__(kBlock) void k_bias_grad(const bf16b *__restrict__ g, int g_c0, int g_ct,
                                                      const bf16b *__restrict__ mask, int mask_c0, int mask_ct,
                                                      int HW, int nsp, double *__restrict__ part) {
    __shared__ double sh[kBlock];
    const int co = blockIdx.x, img = blockIdx.y / nsp, sp = blockIdx.y - img * nsp;
    const int per = (HW + nsp - 1) / nsp, pbeg = sp * per, pend = min(HW, pbeg + per);
    const bf16b *gr = g + ((size_t)img * g_ct + g_c0 + co) * HW;
    const bf16b *mr = mask ? mask + ((size_t)img * mask_ct + mask_c0 + co) * HW : nullptr;
    double s = 0.0;
    for (int p = pbeg + threadIdx.x; p < pend; p += kBlock) {
        float v = b2f(gr[p]);
        if (mr && !(b2f(mr[p]) > 0.0f)) v = 0.0f;
        s += v;
    }
    s = block_sum_256(s, sh);
    if (threadIdx.x == 0) part[(size_t)co * gridDim.y + blockIdx.y] = s;
}

__global__ void k_bias_reduce(const double *__restrict__ part, int nper, int Cout, float *__restrict__ gb) {
    const int co = blockIdx.x * blockDim.x + threadIdx.x;
    if (co >= Cout) return;
    double s = 0.0;
    for (int k = 0; k < nper; ++k) s += part[(size_t)co * nper + k];
    gb[co] = (float)s;
}

// W'[ci][co][ks-1-ky][ks-1-kx] = W[co][ci][ky][kx]
__global__ void k_flip_weights(const bf16b *__restrict__ w, bf16b *__restrict__ wt, int Cout, int Cin, int ks) {
    const int ks2 = ks * ks;
    const size_t n = (size_t)Cout * Cin * ks2;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int kk = (int)(e % ks2);
        const size_t r = e / ks2;
        const int ci = (int)(r % Cin), co = (int)(r / Cin);
        wt[((size_t)ci * Cout + co) * ks2 + (ks2 - 1 - kk)] = w[e];
    }
}

// ---------------------------------------------------------------------------
// elementwise kernels
// ---------------------------------------------------------------------------
// x_bf16 = scale * x (input images to the network)
__global__ void k_to_bf16(const float *__restrict__ x, float scale, bf16b *__restrict__ y, size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        y[e] = f2b(scale * x[e]);
}

// 2x2 average pool of channels [src_c0, src_c0 + C) of src into dst (dense C channels)
__global__ void k_pool_fwd(const bf16b *__restrict__ src, int src_c0, int src_ct, bf16b *__restrict__ dst, int n, int C,
                           int H, int W) {
    const int Ho = H / 2, Wo = W / 2;
    const size_t tot = (size_t)n * C * Ho * Wo;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(e % Wo);
        size_t r = e / Wo;
        const int y = (int)(r % Ho);
        r /= Ho;
        const int c = (int)(r % C), img = (int)(r / C);
        const bf16b *s = src + ((size_t)img * src_ct + src_c0 + c) * H * W;
        const float v = 0.25f * (b2f(s[(2 * y) * W + 2 * x]) + b2f(s[(2 * y) * W + 2 * x + 1]) +
                                 b2f(s[(2 * y + 1) * W + 2 * x]) + b2f(s[(2 * y + 1) * W + 2 * x + 1]));
        dst[e] = f2b(v);
    }
}

// gradient of the pool: dst channels [dst_c0, ...) += g/4 (the skip path wrote there first)
__global__ void k_pool_bwd_add(const bf16b *__restrict__ g, bf16b *__restrict__ dst, int dst_c0, int dst_ct, int n,
                               int C, int H, int W) {
    const size_t tot = (size_t)n * C * H * W;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(e % W);
        size_t r = e / W;
        const int y = (int)(r % H);
        r /= H;
        const int c = (int)(r % C), img = (int)(r / C);
        const float gv = 0.25f * b2f(g[(((size_t)img * C + c) * (H / 2) + y / 2) * (W / 2) + x / 2]);
        bf16b *d = dst + ((size_t)img * dst_ct + dst_c0 + c) * H * W + (size_t)y * W + x;
        *d = f2b(b2f(*d) + gv);
    }
}

// nearest 2x upsample of src (dense C channels, H/2 x W/2) into dst channels [dst_c0, dst_c0 + C)
__global__ void k_up_fwd(const bf16b *__restrict__ src, int src_c0, int src_ct, bf16b *__restrict__ dst, int dst_c0,
                         int dst_ct, int n, int C, int H, int W) {
    const size_t tot = (size_t)n * C * H * W;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(e % W);
        size_t r = e / W;
        const int y = (int)(r % H);
        r /= H;
        const int c = (int)(r % C), img = (int)(r / C);
        dst[((size_t)img * dst_ct + dst_c0 + c) * H * W + (size_t)y * W + x] =
            src[(((size_t)img * src_ct + src_c0 + c) * (H / 2) + y / 2) * (W / 2) + x / 2];
    }
}

// gradient of the upsample: dst (C channels, H/2 x W/2) = sum of the 2x2 block of g channels [g_c0, ...)
__global__ void k_up_bwd(const bf16b *__restrict__ g, int g_c0, int g_ct, bf16b *__restrict__ dst, int dst_c0,
                         int dst_ct, int n, int C, int H, int W) {
    const int Ho = H / 2, Wo = W / 2;
    const size_t tot = (size_t)n * C * Ho * Wo;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(e % Wo);
        size_t r = e / Wo;
        const int y = (int)(r % Ho);
        r /= Ho;
        const int c = (int)(r % C), img = (int)(r / C);
        const bf16b *s = g + ((size_t)img * g_ct + g_c0 + c) * H * W;
        const float v = b2f(s[(2 * y) * W + 2 * x]) + b2f(s[(2 * y) * W + 2 * x + 1]) + b2f(s[(2 * y + 1) * W + 2 * x]) +
                        b2f(s[(2 * y + 1) * W + 2 * x + 1]);
        dst[((size_t)img * dst_ct + dst_c0 + c) * Ho * Wo + (size_t)y * Wo + x] = f2b(v);
    }
}

// loss = mean (out - t)^2 (partials per block, FP64); g = 2 (out - t) / count as BF16 (scaled by gscale)
__global__ __launch_bounds__(kBlock) void k_mse(const float *__restrict__ out, const float *__restrict__ t, size_t n,
                                                float tscale, float gscale, bf16b *__restrict__ g,
                                                double *__restrict__ partial) {
    __shared__ double sh[kBlock];
    double s = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const float d = out[e] - tscale * t[e];
        s += (double)d * d;
        if (g) g[e] = f2b(gscale * 2.0f * d / (float)n);
    }
    s = block_sum_256(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Adam on FP32 master weights; writes the BF16 copy of weight entries (idx < nw)
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       size_t n, float lr, float b1, float b2, float eps, float c1, float c2, float ginv,
                       bf16b *__restrict__ wb, size_t nw) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const float gr = g[e] * ginv;
        const float mm = b1 * m[e] + (1.0f - b1) * gr;
        const float vv = b2 * v[e] + (1.0f - b2) * gr * gr;
        m[e] = mm;
        v[e] = vv;
        const float pv = p[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
        p[e] = pv;
        if (e < nw) wb[e] = f2b(pv);
    }
}

__global__ void k_f32_to_bf16(const float *__restrict__ x, bf16b *__restrict__ y, size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        y[e] = f2b(x[e]);
}

__global__ void k_fill_f32(float *x, size_t n, float v) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) x[e] = v;
}

__global__ void k_fill_bf16(bf16b *x, size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) x[e] = 0;
}

__global__ void k_scale_copy(const float *__restrict__ x, float s, float *__restrict__ y, size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        y[e] = s * x[e];
}

__global__ void k_count_nonfinite(const float *__restrict__ x, size_t n, int *flag) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        if (!isfinite(x[e])) *flag = 1;
}

// Box average over f x f blocks, [nc][H][W] -> [nc][H/f][W/f] (FP32).
__global__ void k_box_down(const float *__restrict__ src, float *__restrict__ dst, size_t nc, int H, int W, int f) {
    const int h = H / f, w = W / f;
    const size_t n = nc * h * w;
    const float inv = 1.0f / (float)(f * f);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(e % w);
        const size_t t = e / w;
        const int y = (int)(t % h);
        const size_t c = t / h;
        const float *s = src + (c * H + (size_t)y * f) * W + (size_t)x * f;
        float acc = 0.0f;
        for (int dy = 0; dy < f; ++dy)
            for (int dx = 0; dx < f; ++dx) acc += s[(size_t)dy * W + dx];
        dst[e] = acc * inv;
    }
}

// Bilinear upsampling by f with pixel centres aligned: output pixel X samples
// the source at (X + 1/2) / f - 1/2, clamped to the first and last pixel.
__global__ void k_bilinear_up(const float *__restrict__ src, float *__restrict__ dst, size_t nc, int h, int w,
                              int f) {
    const int H = h * f, W = w * f;
    const size_t n = nc * H * W;
    const float invf = 1.0f / (float)f;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int X = (int)(e % W);
        const size_t t = e / W;
        const int Y = (int)(t % H);
        const size_t c = t / H;
        const float sy = fmaxf(((float)Y + 0.5f) * invf - 0.5f, 0.0f);
        const float sx = fmaxf(((float)X + 0.5f) * invf - 0.5f, 0.0f);
        const int y0 = min((int)sy, h - 1), x0 = min((int)sx, w - 1);
        const int y1 = min(y0 + 1, h - 1), x1 = min(x0 + 1, w - 1);
        const float ay = sy - (float)y0, ax = sx - (float)x0;
        const float *s = src + c * h * w;
        const float top = (1.0f - ax) * s[y0 * w + x0] + ax * s[y0 * w + x1];
        const float bot = (1.0f - ax) * s[y1 * w + x0] + ax * s[y1 * w + x1];
        dst[e] = (1.0f - ay) * top + ay * bot;
    }
}

static int eblocks(size_t n) { return (int)std::max<size_t>(1, std::min<size_t>((n + kBlock - 1) / kBlock, 8192)); }

// ---- launchers used by the host-side network
void cnn_conv_fwd(const ConvFwd &a, hipStream_t st) {
    dim3 grid((a.H * a.W + kT - 1) / kT, (a.Cout + kT - 1) / kT, a.n);
    if (a.ks == 3) k_conv_fwd<3><<<grid, kBlock, 0, st>>>(a);
    else if (a.ks == 1) k_conv_fwd<1><<<grid, kBlock, 0, st>>>(a);
    else k_conv_fwd<0><<<grid, kBlock, 0, st>>>(a);
}
void cnn_conv_wgrad(const ConvWgrad &a, hipStream_t st) {
    const int K = a.Cin * a.ks * a.ks;
    dim3 grid((K + kT - 1) / kT, (a.Cout + kT - 1) / kT, a.nsplit);
    if (a.ks == 3) k_conv_wgrad<3><<<grid, kBlock, 0, st>>>(a);
    else if (a.ks == 1) k_conv_wgrad<1><<<grid, kBlock, 0, st>>>(a);
    else k_conv_wgrad<0><<<grid, kBlock, 0, st>>>(a);
}
void cnn_wgrad_reduce(const float *partial, int nsplit, size_t n, float *gw, hipStream_t st) {
    k_wgrad_reduce<<<eblocks(n), kBlock, 0, st>>>(partial, nsplit, n, gw);
}
int cnn_bias_splits(int n, int HW, int Cout) {
    // pixel ranges per image: about 2048 blocks in all, at least 1024 pixels each
    int nsp = std::max(1, 2048 / std::max(1, Cout * n));
    return std::min(nsp, std::max(1, HW / 1024));
}
void cnn_bias_grad(const bf16b *g, int g_c0, int g_ct, const bf16b *mask, int mask_c0, int mask_ct, int n, int HW,
                   int Cout, double *part, float *gb, hipStream_t st) {
    const int nsp = cnn_bias_splits(n, HW, Cout);
    k_bias_grad<<<dim3(Cout, n * nsp), kBlock, 0, st>>>(g, g_c0, g_ct, mask, mask_c0, mask_ct, HW, nsp, part);
    k_bias_reduce<<<(Cout + kBlock - 1) / kBlock, kBlock, 0, st>>>(part, n * nsp, Cout, gb);
}
void cnn_flip(const bf16b *w, bf16b *wt, int Cout, int Cin, int ks, hipStream_t st) {
    k_flip_weights<<<eblocks((size_t)Cout * Cin * ks * ks), kBlock, 0, st>>>(w, wt, Cout, Cin, ks);
}
void cnn_to_bf16(const float *x, float s, bf16b *y, size_t n, hipStream_t st) {
    k_to_bf16<<<eblocks(n), kBlock, 0, st>>>(x, s, y, n);
}
void cnn_pool_fwd(const bf16b *src, int c0, int ct, bf16b *dst, int n, int C, int H, int W, hipStream_t st) {
    k_pool_fwd<<<eblocks((size_t)n * C * H * W / 4), kBlock, 0, st>>>(src, c0, ct, dst, n, C, H, W);
}
void cnn_pool_bwd_add(const bf16b *g, bf16b *dst, int c0, int ct, int n, int C, int H, int W, hipStream_t st) {
    k_pool_bwd_add<<<eblocks((size_t)n * C * H * W), kBlock, 0, st>>>(g, dst, c0, ct, n, C, H, W);
}
void cnn_up_fwd(const bf16b *src, int sc0, int sct, bf16b *dst, int dc0, int dct, int n, int C, int H, int W,
                hipStream_t st) {
    k_up_fwd<<<eblocks((size_t)n * C * H * W), kBlock, 0, st>>>(src, sc0, sct, dst, dc0, dct, n, C, H, W);
}
void cnn_up_bwd(const bf16b *g, int gc0, int gct, bf16b *dst, int dc0, int dct, int n, int C, int H, int W,
                hipStream_t st) {
    k_up_bwd<<<eblocks((size_t)n * C * H * W / 4), kBlock, 0, st>>>(g, gc0, gct, dst, dc0, dct, n, C, H, W);
}
int cnn_mse(const float *out, const float *t, size_t n, float tscale, float gscale, bf16b *g, double *partial,
            hipStream_t st) {
    const int nb = std::min(eblocks(n), 1024);
    k_mse<<<nb, kBlock, 0, st>>>(out, t, n, tscale, gscale, g, partial);
    return nb;
}
void cnn_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2, float eps, float c1,
              float c2, float ginv, bf16b *wb, size_t nw, hipStream_t st) {
    k_adam<<<eblocks(n), kBlock, 0, st>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2, ginv, wb, nw);
}
void cnn_f32_to_bf16(const float *x, bf16b *y, size_t n, hipStream_t st) {
    k_f32_to_bf16<<<eblocks(n), kBlock, 0, st>>>(x, y, n);
}
void cnn_fill_f32(float *x, size_t n, float v, hipStream_t st) { k_fill_f32<<<eblocks(n), kBlock, 0, st>>>(x, n, v); }
void cnn_fill_bf16(bf16b *x, size_t n, hipStream_t st) { k_fill_bf16<<<eblocks(n), kBlock, 0, st>>>(x, n); }
void cnn_scale_copy(const float *x, float s, float *y, size_t n, hipStream_t st) {
    k_scale_copy<<<eblocks(n), kBlock, 0, st>>>(x, s, y, n);
}
void cnn_box_down(const float *src, float *dst, size_t nc, int H, int W, int f, hipStream_t st) {
    k_box_down<<<eblocks(nc * (H / f) * (W / f)), kBlock, 0, st>>>(src, dst, nc, H, W, f);
}
void cnn_bilinear_up(const float *src, float *dst, size_t nc, int h, int w, int f, hipStream_t st) {
    k_bilinear_up<<<eblocks(nc * h * w * f * f), kBlock, 0, st>>>(src, dst, nc, h, w, f);
}
void cnn_count_nonfinite(const float *x, size_t n, int *flag, hipStream_t st) {
    k_count_nonfinite<<<eblocks(n), kBlock, 0, st>>>(x, n, flag);
}

}  // namespace tnlm
