// TNLM regulariser with the patch distances of Eq. 8 recast as a dense
// contraction on the BF16 matrix cores (ssd_mode = TNLM_SSD_BF16_MFMA):
//   D(x, y) = ||a||^2 + ||b||^2 - 2 <a, b>,  a = patch of x in g_i, b = patch of y in g_j.
// The cross terms <a, b> for 16 outputs of one image row against the 32
// candidate columns of one window row come from v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation. Compensation: (i) every value is centred on a per-tile
// reference (the distance is shift invariant) so the products are small;
// (ii) each centred FP32 value is split into BF16 hi + lo and the cross term
// is hi*hi + hi*lo + lo*hi (three MFMAs); (iii) the norms are FP32 sums of
// the centred values; (iv) D is clamped at 0. The exponentials, the running
// normalisation and the Gauss-Jacobi update (Eq. 7) stay in FP32, as in the
// FP32 kernel.
//
// MFMA operand layout (16x16x32, 64 lanes): lane l holds 8 consecutive K
// values k = 8*(l/16) + [0, 8) of row (A) / column (B) l % 16; the result
// holds rows 4*(l/16) + [0, 4) of column l % 16. K = (patch row py, patch
// column px) with px padded to 8: two K-chunks of 4 patch rows each (patch
// sizes 3, 5, 7). A is zero at padded (py, px); the B values there are
// finite tile values and do not contribute.
//
// Tile: 16 x 16 outputs of one phase per 256-thread block; wave w owns output
// rows 4w .. 4w+3, one at a time. Each neighbour tile is read from memory
// once and written to LDS as BF16 hi and lo planes in 8 copies shifted by
// 0..7 elements, so each lane's 8 consecutive values are one aligned 16-byte
// read, and in FP32; the patch norms of the candidates (and of the outputs,
// from the staged own tile) are box sums over those FP32 tiles.
#include "devutil.h"
#include "internal.h"

namespace tnlm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr int kMT = 16;        // output tile side
constexpr int kRowW = 48;      // LDS row width (elements) of a shifted copy
constexpr int kMaxR = 7;       // window radius supported by the MFMA kernel (W <= 15)

struct RegMfmaArgs {
    int R;
    float nk, cs, cn;
    const float *guide, *value, *g;
    float *out;
    int clamp;
    double *relpart;
    int *nonfinite;
};

__device__ __forceinline__ unsigned short bf16_bits(float x) {
    const __bf16 h = (__bf16)x;   // round to nearest even
    return __builtin_bit_cast(unsigned short, h);
}

__device__ __forceinline__ float bf16_to_f(unsigned short b) {
    return __builtin_bit_cast(float, (unsigned)b << 16);
}

__device__ __forceinline__ void online_add_m(float D, float v, float nk, float &Dm, float &num, float &den) {
    if (D < Dm) {
        const float sc = __builtin_amdgcn_exp2f((Dm - D) * nk);
        num *= sc;
        den *= sc;
        Dm = D;
    }
    const float w = __builtin_amdgcn_exp2f((D - Dm) * nk);
    num = fmaf(w, v, num);
    den += w;
}

__device__ __forceinline__ void merge_m(float nk, float Dm1, float num1, float den1, float &Dm, float &num,
                                        float &den) {
    if (!(Dm1 < INFINITY)) return;    // other partial is empty
    if (!(Dm < INFINITY)) {           // this partial is empty
        Dm = Dm1;
        num = num1;
        den = den1;
        return;
    }
    const float m = fminf(Dm, Dm1);
    const float s0 = __builtin_amdgcn_exp2f((Dm - m) * nk);
    const float s1 = __builtin_amdgcn_exp2f((Dm1 - m) * nk);
    num = num * s0 + num1 * s1;
    den = den * s0 + den1 * s1;
    Dm = m;
}

// Sums of squares of the d x d patches of a staged tile: hs[r][c] = sum over
// px of t[r][c + px]^2 (r < rows, c < cols), then out[r][c] = sum over py of
// hs[r + py][c] (r < rows - d + 1); fixed order, one pass each.
template <int d>
__device__ void patch_norms(const float *t, int tw, int rows, int cols, float *hs, float *out) {
    for (int e = threadIdx.x; e < rows * cols; e += kBlock) {
        const int r = e / cols, c = e - r * cols;
        float s2 = 0.0f;
#pragma unroll
        for (int px = 0; px < d; ++px) {
            const float v = t[r * tw + c + px];
            s2 = fmaf(v, v, s2);
        }
        hs[e] = s2;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < (rows - d + 1) * cols; e += kBlock) {
        const int r = e / cols, c = e - r * cols;
        float s2 = 0.0f;
#pragma unroll
        for (int py = 0; py < d; ++py) s2 += hs[(r + py) * cols + c];
        out[e] = s2;
    }
    __syncthreads();
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_tnlm_reg_mfma(Batch bt, Stage st, RegMfmaArgs a) {
    constexpr int d = 2 * S + 1;
    constexpr int OT = kMT + 2 * S;            // own tile side (outputs and patch halo)
    extern __shared__ unsigned char smem[];
    const int R = a.R;
    const int TR = kMT + 2 * R + 8;            // tile rows (window + patch rows padded to 8)
    const int plane = TR * kRowW;              // elements of one shifted copy
    const int NC = kMT + 2 * R;                // candidate region side
    const int NT = NC + 2 * S;                 // neighbour tile side (candidates and patch halo)
    unsigned short *hi = (unsigned short *)smem;          // [8][TR][kRowW]
    unsigned short *lo = hi + 8 * plane;                   // [8][TR][kRowW]
    float *nrm = (float *)(lo + 8 * plane);                // candidate norms [NC][NC]
    float *ft = nrm + NC * NC;                             // centred FP32 tile [NT][NT] (own: [OT][OT])
    float *hs = ft + NT * NT;                              // row sums of squares [NT][NC]
    float *nown = hs + NT * NC;                            // norms of the tile's outputs [kMT][kMT]
    float *oacc = nown + kMT * kMT;                        // sum over neighbours of A_j per output [kMT][kMT]
    float *fo = oacc + kMT * kMT;                          // own tile, centred [OT][OT]
    float *vt = fo + OT * OT;                              // the neighbour's values at the candidates [NC][NC]
    __shared__ double shred[kBlock];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n16 = lane & 15, kg = lane >> 4;

    __shared__ int sh_item;
    WorkIter it = work_begin(st);
    int gb;
    while (work_next(st, it, gb, &sh_item)) {
        const int sidx = find_slice(st.pre, bt.ns, gb);
        if (bt.skip && bt.skip[sidx]) continue;
        const SliceDesc sd = bt.sl[sidx];
        const int L = sd.L, N = sd.N;
        const int nt = (L + kMT - 1) / kMT;
        const int lb = gb - st.pre[sidx];
        const int tl = lb % (nt * nt), i = lb / (nt * nt);
        const int x0 = (tl % nt) * kMT, y0 = (tl / nt) * kMT;
        const size_t pl = (size_t)L * L;
        const float *gimg = a.guide + sd.img0;
        const float *vimg = a.value + sd.img0;
        const float *gi = gimg + (size_t)i * pl;
        // centring reference: the guide value at the tile's first pixel
        const float c0 = gi[(size_t)y0 * L + x0];

        // own tile, centred, edge-clamped: the outputs' patch values once from
        // memory; their norms by box sums; the A operands from LDS
        __syncthreads();   // LDS reuse across work items
        for (int e = threadIdx.x; e < OT * OT; e += kBlock) {
            const int r = e / OT, c = e - r * OT;
            const int gr = min(max(y0 - S + r, 0), L - 1), gc = min(max(x0 - S + c, 0), L - 1);
            fo[e] = gi[(size_t)gr * L + gc] - c0;
        }
        for (int e = threadIdx.x; e < kMT * kMT; e += kBlock) oacc[e] = 0.0f;
        __syncthreads();
        patch_norms<d>(fo, OT, OT, kMT, hs, nown);

        for (int nb = 0; nb < 2; ++nb) {
            const int j = nb == 0 ? (i - 1 + N) % N : (i + 1) % N;
            const float *gj = gimg + (size_t)j * pl;
            const float *vj = vimg + (size_t)j * pl;
            const int row0 = y0 - R - S, col0 = x0 - R - S;
            __syncthreads();   // LDS reuse (own tile, previous neighbour)
            // stage the neighbour tile: centred values split to hi/lo in 8
            // shifted copies (each lane's 8 consecutive values are one aligned
            // read), and in FP32 for the norms; one read from memory each
            for (int e = threadIdx.x; e < TR * kRowW; e += kBlock) {
                const int tr = e / kRowW, tc = e - tr * kRowW;
                const int r = min(max(row0 + tr, 0), L - 1), c = min(max(col0 + tc, 0), L - 1);
                const float v = gj[(size_t)r * L + c] - c0;
                const unsigned short hb = bf16_bits(v);
                const unsigned short lb2 = bf16_bits(v - bf16_to_f(hb));
#pragma unroll
                for (int sft = 0; sft < 8; ++sft) {
                    const int dst = tc - sft;   // copy sft holds element (tr, tc) at column tc - sft
                    if (dst >= 0) {
                        hi[sft * plane + tr * kRowW + dst] = hb;
                        lo[sft * plane + tr * kRowW + dst] = lb2;
                    }
                }
                if (tr < NT && tc < NT) ft[tr * NT + tc] = v;
            }
            for (int e = threadIdx.x; e < NC * NC; e += kBlock) {
                const int cr = e / NC, cc = e - cr * NC;
                const int r = min(max(y0 - R + cr, 0), L - 1), c = min(max(x0 - R + cc, 0), L - 1);
                vt[e] = vj[(size_t)r * L + c];
            }
            __syncthreads();
            patch_norms<d>(ft, NT, NT, NC, hs, nrm);

#pragma unroll 1
            for (int rr = 0; rr < 4; ++rr) {
                const int yo = y0 + 4 * wave + rr;
                // A operands (own phase) of this output row: hi/lo x 2 K-chunks
                bf16x8 Ahi[2], Alo[2];
#pragma unroll
                for (int kc = 0; kc < 2; ++kc) {
                    const int py = 4 * kc + kg;
                    us8 h, l;
#pragma unroll
                    for (int px = 0; px < 8; ++px) {
                        const float v = (py < d && px < d) ? fo[(4 * wave + rr + py) * OT + n16 + px] : 0.0f;
                        const unsigned short hb = bf16_bits(v);
                        h[px] = hb;
                        l[px] = bf16_bits(v - bf16_to_f(hb));
                    }
                    Ahi[kc] = __builtin_bit_cast(bf16x8, h);
                    Alo[kc] = __builtin_bit_cast(bf16x8, l);
                }
                float na[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) na[t] = nown[(4 * wave + rr) * kMT + 4 * kg + t];
                float Dm[4], num[4], den[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    Dm[t] = INFINITY;
                    num[t] = den[t] = 0.0f;
                }
#pragma unroll 1
                for (int dy = -R; dy <= R; ++dy) {
                    const int cy = yo + dy;             // candidate row
                    const int crow = 4 * wave + rr + dy + R;   // candidate row within the tile region
                    // the two candidate blocks' products, interleaved so that each
                    // MFMA waits on the one two back
                    floatx4 C[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
                    bf16x8 Bh[2][2], Bl[2][2];
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int ncol = 16 * h2 + n16;        // candidate column within the region
                        const int sft = ncol & 7, base = ncol - sft;
#pragma unroll
                        for (int kc = 0; kc < 2; ++kc) {
                            const int tr = crow + 4 * kc + kg;  // tile row of patch row py = 4kc + kg
                            Bh[h2][kc] = __builtin_bit_cast(bf16x8, *(const us8 *)(hi + sft * plane + tr * kRowW + base));
                            Bl[h2][kc] = __builtin_bit_cast(bf16x8, *(const us8 *)(lo + sft * plane + tr * kRowW + base));
                        }
                    }
#pragma unroll
                    for (int kc = 0; kc < 2; ++kc) {
#pragma unroll
                        for (int h2 = 0; h2 < 2; ++h2)
                            C[h2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahi[kc], Bh[h2][kc], C[h2], 0, 0, 0);
#pragma unroll
                        for (int h2 = 0; h2 < 2; ++h2)
                            C[h2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahi[kc], Bl[h2][kc], C[h2], 0, 0, 0);
#pragma unroll
                        for (int h2 = 0; h2 < 2; ++h2)
                            C[h2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Alo[kc], Bh[h2][kc], C[h2], 0, 0, 0);
                    }
                    if ((unsigned)cy >= (unsigned)L) continue;
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int ncol = 16 * h2 + n16;
                        const int cx = x0 - R + ncol;   // candidate column
                        const bool colok = (unsigned)cx < (unsigned)L && ncol < NC;
                        const float nbv = colok ? nrm[crow * NC + ncol] : 0.0f;
                        const float vv = colok ? vt[crow * NC + ncol] : 0.0f;
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int m = 4 * kg + t;          // output column within the tile
                            const int dx = ncol - R - m;
                            if (!colok || dx < -R || dx > R) continue;
                            const float D = fmaxf(fmaf(-2.0f, C[h2][t], na[t] + nbv), 0.0f);
                            online_add_m(D, vv, a.nk, Dm[t], num[t], den[t]);
                        }
                    }
                }
                // merge the 16 lanes holding the same outputs (different candidates)
#pragma unroll
                for (int off = 1; off < 16; off <<= 1)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float Dm1 = __shfl_xor(Dm[t], off, 64);
                        const float n1 = __shfl_xor(num[t], off, 64);
                        const float d1 = __shfl_xor(den[t], off, 64);
                        merge_m(a.nk, Dm1, n1, d1, Dm[t], num[t], den[t]);
                    }
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (n16 == 0) oacc[(4 * wave + rr) * kMT + 4 * kg + t] += num[t] / den[t];
            }
        }

        // epilogue: lane n16 == 0 of each 16-lane group writes its 4 outputs per row
        double dd = 0.0, nn = 0.0;
        bool bad = false;
        if (n16 == 0) {
            const float *gl = a.g + sd.img0 + (size_t)i * pl;
            float *oi = a.out + sd.img0 + (size_t)i * pl;
            for (int rr = 0; rr < 4; ++rr) {
                const int yo = y0 + 4 * wave + rr;
                if (yo >= L) continue;
                for (int t = 0; t < 4; ++t) {
                    const int xo = x0 + 4 * kg + t;
                    if (xo >= L) continue;
                    const size_t e = (size_t)yo * L + xo;
                    float u = fmaf(a.cn, oacc[(4 * wave + rr) * kMT + 4 * kg + t], a.cs * gl[e]);
                    if (a.clamp) u = fmaxf(u, 0.0f);
                    if (a.relpart) {
                        const double df = (double)u - (double)oi[e];
                        dd += df * df;
                        nn += (double)u * (double)u;
                    }
                    bad |= !isfinite(u);
                    oi[e] = u;
                }
            }
        }
        if (bad && a.nonfinite) a.nonfinite[sidx] = 1;
        if (a.relpart) {
            dd = block_sum_256(dd, shred);
            nn = block_sum_256(nn, shred);
            if (threadIdx.x == 0) {
                a.relpart[2 * ((long long)sd.rp0 + lb)] = dd;
                a.relpart[2 * ((long long)sd.rp0 + lb) + 1] = nn;
            }
        }
    }
    work_end(st);
}

int reg_mfma_blocks(const SliceDesc &s) {
    const int t = (s.L + kMT - 1) / kMT;
    return t * t * s.N;
}

bool reg_mfma_supported(int patch, int window) {
    return (patch == 3 || patch == 5 || patch == 7) && window >= 3 && window <= 2 * kMaxR + 1 && (window & 1);
}

static size_t mfma_lds_bytes(int R, int S) {
    const int TR = kMT + 2 * R + 8, NC = kMT + 2 * R, NT = NC + 2 * S;
    const int OT = kMT + 2 * S;
    return (size_t)2 * 8 * TR * kRowW * sizeof(unsigned short) +
           (2 * (size_t)NC * NC + (size_t)NT * NT + (size_t)NT * NC + 2 * kMT * kMT + (size_t)OT * OT) * sizeof(float);
}

void launch_regularize_mfma(const Batch &b, const Stage &st, const RegParams &p, const float *guide,
                            const float *value, const float *g, float *out, int clamp, double *relpart,
                            int *nonfinite, hipStream_t strm) {
    if (st.total == 0) return;
    RegMfmaArgs a;
    a.R = p.window / 2;
    a.nk = (float)(-1.4426950408889634 / ((double)p.h * (double)p.h));
    a.cs = (float)(1.0 / (1.0 + (double)p.mu_hat));
    a.cn = (float)((double)p.mu_hat / (2.0 * (double)p.mu_hat + 2.0));
    a.guide = guide;
    a.value = value;
    a.g = g;
    a.out = out;
    a.clamp = clamp;
    a.relpart = relpart;
    a.nonfinite = nonfinite;
    const size_t lds = mfma_lds_bytes(a.R, p.patch / 2);
    switch (p.patch / 2) {
        case 1: k_tnlm_reg_mfma<1><<<st.grid, kBlock, lds, strm>>>(b, st, a); break;
        case 2: k_tnlm_reg_mfma<2><<<st.grid, kBlock, lds, strm>>>(b, st, a); break;
        default: k_tnlm_reg_mfma<3><<<st.grid, kBlock, lds, strm>>>(b, st, a); break;
    }
}

}  // namespace tnlm
