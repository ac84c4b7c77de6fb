// TNLM regulariser: Eq. 8 patch weights over the §2.3 search window of the two
// neighbouring phases, fused with one Gauss-Jacobi sweep of Eq. 7 and the
// positivity clamp of the TNLM algorithm box:
//   out_i(x) = g_i(x)/(1+mu) + mu/(2mu+2) * sum_{j = i-1, i+1} A_j(x),
//   A_j(x)   = sum_y w_ij(x,y) value_j(y) / sum_y w_ij(x,y),
//   w_ij     = exp(-(D(x,y) - min_y D)/h^2),  D = SSD of d x d guide patches,
// with y over the W x W window truncated to the image and patch pixels outside
// the image replaced by the nearest edge pixel.
//
// CDNA4 mapping (one 256-thread block per output tile of 4*BY rows x (32-2S)
// columns of one phase; S = (d-1)/2, R = (W-1)/2, BY = output rows per lane;
// blocks loop persistently over the tiles of every slice of a batch):
//   * guide/value tiles of both neighbour phases, with the window and patch
//     halo, are staged once in LDS (edge-clamped at load time);
//   * wave w handles neighbour j = w & 1 and half of the window rows
//     (dy <= 0 or dy > 0); its 64 lanes are 4 rows of 16 lanes, each lane
//     owns 2 adjacent columns and 8 output rows;
//   * per offset (dx, dy) a lane forms the squared differences E of its
//     columns over BY + 2S rows against its own phase's values held in
//     registers, sums them down the patch rows in registers and then, for its
//     BY output rows, across the patch columns with DPP row shifts (16-lane
//     rows, (32-2S)/32 of the lanes produce valid columns) -- all sums are of
//     non-negative terms, no sliding subtraction;
//   * the weights are accumulated with a running minimum distance (online
//     normalisation: a new minimum rescales the running sums), so each pair
//     costs one exp2 and the result equals Eq. 8 with the window-minimum shift;
//   * the two window halves and the two neighbours are merged through LDS;
//     the epilogue applies Eq. 7, the clamp, and emits the partial sums of the
//     relative update ||f_new - f_old||, ||f_new|| when asked.
#include "devutil.h"
#include "internal.h"

namespace tnlm {

struct RegArgs {
    int R;
    float nk;        // -log2(e) / h^2
    float cs, cn;    // 1/(1+mu), mu/(2mu+2)
    const float *guide, *value, *g;
    float *out;
    int clamp;
    double *relpart;
    int *nonfinite;  // [ns]
};

// Value of x held by lane (l + K) of the same 16-lane row; 0 outside the row.
template <int K>
__device__ __forceinline__ float rowsh(float x) {
    if constexpr (K == 0) {
        return x;
    } else if constexpr (K > 0) {
        return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x100 + K, 0xF,
                                                                     0xF, true));   // row_shl:K
    } else {
        return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x110 - K, 0xF,
                                                                     0xF, true));   // row_shr:-K
    }
}

template <int K0, int K1>
__device__ __forceinline__ float rowsum(float x) {
    if constexpr (K0 > K1) return 0.0f;
    else if constexpr (K0 == K1) return rowsh<K0>(x);
    else return rowsh<K0>(x) + rowsum<K0 + 1, K1>(x);
}

// Patch-row sums for the lane's two columns xa = base + 2l (value ea) and
// xb = xa + 1 (value eb), given p = ea + eb: ha = sum of E over columns
// xa-S..xa+S, hb over xb-S..xb+S.
template <int S>
__device__ __forceinline__ void hsum(float ea, float eb, float p, float &ha, float &hb) {
    if constexpr (S % 2 == 1) {
        constexpr int H = (S - 1) / 2;
        const float qs = rowsum<-H, H>(p);
        ha = qs + rowsh<-(S + 1) / 2>(eb);
        hb = qs + rowsh<(S + 1) / 2>(ea);
    } else {
        constexpr int H = S / 2;
        ha = rowsum<-H, H - 1>(p) + rowsh<H>(ea);
        hb = rowsh<-H>(eb) + rowsum<-H + 1, H>(p);
    }
}

template <int S>
__device__ __forceinline__ bool lane_valid_a(int l) {
    if constexpr (S % 2 == 1) return l >= (S + 1) / 2 && l + (S - 1) / 2 <= 15;
    else return l >= S / 2 && l + S / 2 <= 15;
}
template <int S>
__device__ __forceinline__ bool lane_valid_b(int l) {
    if constexpr (S % 2 == 1) return l >= (S - 1) / 2 && l + (S + 1) / 2 <= 15;
    else return l >= S / 2 && l + S / 2 <= 15;
}

__device__ __forceinline__ void online_add(float D, float v, float nk, float &Dm, float &num, float &den) {
    if (D < Dm) {   // new window minimum: rescale the running sums
        const float sc = __builtin_amdgcn_exp2f((Dm - D) * nk);
        num *= sc;
        den *= sc;
        Dm = D;
    }
    const float w = __builtin_amdgcn_exp2f((D - Dm) * nk);
    num = fmaf(w, v, num);
    den += w;
}

__device__ __forceinline__ void merge(float nk, float Dm1, float num1, float den1, float &Dm, float &num, float &den) {
    const float m = fminf(Dm, Dm1);
    const float s0 = __builtin_amdgcn_exp2f((Dm - m) * nk);
    const float s1 = __builtin_amdgcn_exp2f((Dm1 - m) * nk);
    num = fmaf(num, s0, num1 * s1);
    den = fmaf(den, s0, den1 * s1);
    Dm = m;
}

template <int S, int kBY>
__global__ __launch_bounds__(kBlock) void k_tnlm_reg(Batch bt, Stage st, RegArgs a) {
    // no implicit multiply-add fusion: whether the compiler fuses would differ
    // between instances of this template, and with it the rounding; every
    // fused operation is written out, so all tile heights give the same bits
#pragma clang fp contract(off)
    extern __shared__ float lds[];
    __shared__ double shred[kBlock];
    constexpr int TW = 32 - 2 * S, TH = 4 * kBY, NR = kBY + 2 * S;
    const int R = a.R;
    const int TCW = 32 + 2 * R, TRH = TH + 2 * S + 2 * R, TS = TCW * TRH;
    const bool same = a.value == a.guide;
    __shared__ int sh_item;
    WorkIter it = work_begin(st);
    int gb;
    while (work_next(st, it, gb, &sh_item)) {
    const int sidx = find_slice(st.pre, bt.ns, gb);
    if (bt.skip && bt.skip[sidx]) continue;
    const SliceDesc sd = bt.sl[sidx];
    const int L = sd.L, N = sd.N;
    const int ntx = (L + TW - 1) / TW, nty = (L + TH - 1) / TH;
    int lb = gb - st.pre[sidx];
    const int tile_local = lb % (ntx * nty);
    const int i = lb / (ntx * nty);
    const int x0 = (tile_local % ntx) * TW, y0 = (tile_local / ntx) * TH;
    const int nbr0 = (i - 1 + N) % N, nbr1 = (i + 1) % N;
    const size_t plane = (size_t)L * L;
    const float *guide = a.guide + sd.img0, *value = a.value + sd.img0;

    __syncthreads();   // LDS reuse across work items
    float *tg0 = lds, *tg1 = lds + TS;
    float *tv0 = same ? tg0 : lds + 2 * TS, *tv1 = same ? tg1 : lds + 3 * TS;
    const int col0 = x0 - S - R, row0 = y0 - S - R;
    for (int e = threadIdx.x; e < TS; e += kBlock) {
        const int tr = e / TCW, tc = e - tr * TCW;
        const int gr = min(max(row0 + tr, 0), L - 1), gc = min(max(col0 + tc, 0), L - 1);
        const size_t off = (size_t)gr * L + gc;
        tg0[e] = guide[nbr0 * plane + off];
        tg1[e] = guide[nbr1 * plane + off];
        if (!same) {
            tv0[e] = value[nbr0 * plane + off];
            tv1[e] = value[nbr1 * plane + off];
        }
    }

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nsel = wave & 1, half = wave >> 1;
    const int l16 = lane & 15, band = lane >> 4;
    const int xa = x0 - S + 2 * l16;
    const int zbase = y0 + band * kBY - S;

    float gia[NR], gib[NR];
    {
        const float *gi = guide + (size_t)i * plane;
        const int ca = min(max(xa, 0), L - 1), cb = min(max(xa + 1, 0), L - 1);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int zr = min(max(zbase + k, 0), L - 1);
            gia[k] = gi[(size_t)zr * L + ca];
            gib[k] = gi[(size_t)zr * L + cb];
        }
    }
    const bool va = lane_valid_a<S>(l16) && xa >= x0 && xa < x0 + TW && xa < L;
    const bool vb = lane_valid_b<S>(l16) && xa + 1 >= x0 && xa + 1 < x0 + TW && xa + 1 < L;

    float Dma[kBY], numa[kBY], dena[kBY], Dmb[kBY], numb[kBY], denb[kBY];
#pragma unroll
    for (int o = 0; o < kBY; ++o) {
        Dma[o] = Dmb[o] = INFINITY;
        numa[o] = dena[o] = numb[o] = denb[o] = 0.0f;
    }
    __syncthreads();

    const float *TG = nsel ? tg1 : tg0;
    const float *TV = nsel ? tv1 : tv0;
    const int ta = 2 * l16 + R;
    const int trb = band * kBY + R;
    const float nk = a.nk;
    const int yb = y0 + band * kBY;

    // offsets nearest the centre first (rows 0, -1, ..., -R for one half and
    // 1, ..., R for the other; columns 0, 1, -1, 2, -2, ...): the smallest
    // distance, usually near the centre, is met early and later offsets
    // rarely rescale the running sums
    const int nrow = half == 0 ? R + 1 : R;
    for (int kr = 0; kr < nrow; ++kr) {
        const int dy = half == 0 ? -kr : kr + 1;
        for (int kc = 0; kc <= 2 * R; ++kc) {
            const int dx = (kc & 1) ? (kc + 1) >> 1 : -(kc >> 1);
            // squared differences of the lane's two columns, summed down the
            // patch rows first, then across the patch columns (DPP) for the
            // BY output rows only
            float ea[NR], eb[NR];
            const float *rowp = TG + (trb + dy) * TCW + ta + dx;
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                const float da = gia[k] - rowp[k * TCW];
                const float db = gib[k] - rowp[k * TCW + 1];
                ea[k] = da * da;
                eb[k] = db * db;
            }
            const bool ca = va && (unsigned)(xa + dx) < (unsigned)L;
            const bool cb = vb && (unsigned)(xa + 1 + dx) < (unsigned)L;
            const float *vp = TV + (band * kBY + S + R + dy) * TCW + ta + dx;
            float p2a[NR - 1], p2b[NR - 1];
#pragma unroll
            for (int k = 0; k + 1 < NR; ++k) {
                p2a[k] = ea[k] + ea[k + 1];
                p2b[k] = eb[k] + eb[k + 1];
            }
#pragma unroll
            for (int o = 0; o < kBY; ++o) {
                float Va = ea[o + 2 * S], Vb = eb[o + 2 * S];
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    Va += p2a[o + 2 * j];
                    Vb += p2b[o + 2 * j];
                }
                float Da, Db;
                hsum<S>(Va, Vb, Va + Vb, Da, Db);
                const bool rv = (unsigned)(yb + o + dy) < (unsigned)L;
                if (rv && ca) online_add(Da, vp[o * TCW], nk, Dma[o], numa[o], dena[o]);
                if (rv && cb) online_add(Db, vp[o * TCW + 1], nk, Dmb[o], numb[o], denb[o]);
            }
        }
    }

    // ---- merge the two window halves (waves 2,3 -> waves 0,1), then the two neighbours
    __syncthreads();   // tiles no longer needed
    float *mrg = lds;  // [2][64][2*kBY][3]
    if (half == 1) {
        float *p = mrg + ((size_t)(nsel * 64 + lane) * 2 * kBY) * 3;
#pragma unroll
        for (int o = 0; o < kBY; ++o) {
            p[3 * o + 0] = Dma[o]; p[3 * o + 1] = numa[o]; p[3 * o + 2] = dena[o];
            p[3 * (kBY + o) + 0] = Dmb[o]; p[3 * (kBY + o) + 1] = numb[o]; p[3 * (kBY + o) + 2] = denb[o];
        }
    }
    __syncthreads();
    float Aa[kBY], Ab[kBY];
    if (half == 0) {
        const float *p = mrg + ((size_t)(nsel * 64 + lane) * 2 * kBY) * 3;
#pragma unroll
        for (int o = 0; o < kBY; ++o) {
            merge(nk, p[3 * o + 0], p[3 * o + 1], p[3 * o + 2], Dma[o], numa[o], dena[o]);
            merge(nk, p[3 * (kBY + o) + 0], p[3 * (kBY + o) + 1], p[3 * (kBY + o) + 2], Dmb[o], numb[o], denb[o]);
            Aa[o] = numa[o] / dena[o];
            Ab[o] = numb[o] / denb[o];
        }
    }
    __syncthreads();
    float *ax = lds + 3 * 2 * 64 * 2 * kBY;   // [64][2*kBY]
    if (wave == 1) {
#pragma unroll
        for (int o = 0; o < kBY; ++o) {
            ax[lane * 2 * kBY + o] = Aa[o];
            ax[lane * 2 * kBY + kBY + o] = Ab[o];
        }
    }
    __syncthreads();
    double dd = 0.0, nn = 0.0;
    if (wave == 0) {
        const float *gi = a.g + sd.img0 + (size_t)i * plane;
        float *oi = a.out + sd.img0 + (size_t)i * plane;
        bool bad = false;
#pragma unroll
        for (int o = 0; o < kBY; ++o) {
            const int yo = yb + o;
            if (yo >= L) continue;
            if (va) {
                const size_t e = (size_t)yo * L + xa;
                float u = fmaf(a.cn, Aa[o] + ax[lane * 2 * kBY + o], a.cs * gi[e]);
                if (a.clamp) u = fmaxf(u, 0.0f);
                if (a.relpart) {
                    const double df = (double)u - (double)oi[e];
                    dd = fma(df, df, dd);
                    nn = fma((double)u, (double)u, nn);
                }
                bad |= !isfinite(u);
                oi[e] = u;
            }
            if (vb) {
                const size_t e = (size_t)yo * L + xa + 1;
                float u = fmaf(a.cn, Ab[o] + ax[lane * 2 * kBY + kBY + o], a.cs * gi[e]);
                if (a.clamp) u = fmaxf(u, 0.0f);
                if (a.relpart) {
                    const double df = (double)u - (double)oi[e];
                    dd = fma(df, df, dd);
                    nn = fma((double)u, (double)u, nn);
                }
                bad |= !isfinite(u);
                oi[e] = u;
            }
        }
        if (bad && a.nonfinite) a.nonfinite[sidx] = 1;
    }
    if (a.relpart) {
        dd = block_sum_256(dd, shred);
        nn = block_sum_256(nn, shred);
        if (threadIdx.x == 0) {
            const long long blk = (long long)sd.rp0 + lb;
            a.relpart[2 * blk] = dd;
            a.relpart[2 * blk + 1] = nn;
        }
    }
    }   // work items
    work_end(st);
}

// Regularisation term of Eq. 1 for one slice: the sum over phases i, both
// neighbours j = i-1, i+1, pixels x and the window offsets y inside the
// image of w_ij(x, y) (f_i(x) - f_j(y))^2, with the normalised weights of
// Eq. 8 from the guide stack (edge-clamped patches, window-minimum shift as
// a running minimum). Direct patch sums, one lane per (pixel, neighbour): a
// diagnostic of the cost, not part of a solve. Per-block FP64 sums in part.
__global__ __launch_bounds__(kBlock) void k_reg_cost(int N, int L, int S, int R, float nk,
                                                     const float *__restrict__ guide, const float *__restrict__ f,
                                                     double *__restrict__ part) {
    __shared__ double sh[kBlock];
    const long long plane = (long long)L * L, total = 2LL * N * plane;
    double acc = 0.0;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const int side = (int)(t & 1);
        long long q = t >> 1;
        const int c = (int)(q % L);
        q /= L;
        const int r = (int)(q % L), i = (int)(q / L);
        const int j = side ? (i + 1) % N : (i - 1 + N) % N;
        const float *gi = guide + i * plane, *gj = guide + j * plane, *fj = f + j * plane;
        const float fx = f[i * plane + (long long)r * L + c];
        float Dm = INFINITY, num = 0.0f, den = 0.0f;
        for (int dy = -R; dy <= R; ++dy) {
            const int r2 = r + dy;
            if (r2 < 0 || r2 >= L) continue;
            for (int dx = -R; dx <= R; ++dx) {
                const int c2 = c + dx;
                if (c2 < 0 || c2 >= L) continue;
                float D = 0.0f;
                for (int py = -S; py <= S; ++py) {
                    const int ra = min(max(r + py, 0), L - 1), rb = min(max(r2 + py, 0), L - 1);
                    for (int px = -S; px <= S; ++px) {
                        const int ca = min(max(c + px, 0), L - 1), cb = min(max(c2 + px, 0), L - 1);
                        const float d = gi[(long long)ra * L + ca] - gj[(long long)rb * L + cb];
                        D = fmaf(d, d, D);
                    }
                }
                const float e = fx - fj[(long long)r2 * L + c2];
                online_add(D, e * e, nk, Dm, num, den);
            }
        }
        acc += (double)num / (double)den;
    }
    acc = block_sum_256(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

int launch_reg_cost(int N, int L, int patch, int window, float h, const float *guide, const float *f, double *part,
                    int max_blocks, hipStream_t strm) {
    const long long total = 2LL * N * L * L;
    const int nb = (int)std::max(1LL, std::min((long long)max_blocks, (total + kBlock - 1) / kBlock));
    const float nk = (float)(-1.4426950408889634 / ((double)h * (double)h));
    k_reg_cost<<<nb, kBlock, 0, strm>>>(N, L, patch / 2, window / 2, nk, guide, f, part);
    return nb;
}

static int tile_w(int patch) { return 32 - 2 * (patch / 2); }

int reg_blocks(const SliceDesc &s, int patch, int rows_per_lane) {
    const int tw = tile_w(patch), th = 4 * rows_per_lane;
    return ((s.L + tw - 1) / tw) * ((s.L + th - 1) / th) * s.N;
}

bool reg_supported(int patch, int window) {
    return patch >= 3 && patch <= 9 && (patch & 1) && window >= 3 && window <= 21 && (window & 1);
}

static size_t reg_lds_bytes(const RegParams &p, int BY, bool same) {
    const int S = p.patch / 2, R = p.window / 2;
    const size_t ts = (size_t)(32 + 2 * R) * (4 * BY + 2 * S + 2 * R);
    const size_t tiles = (same ? 2 : 4) * ts;
    const size_t merge = 3 * 2 * 64 * 2 * BY + 64 * 2 * BY;
    return std::max(tiles, merge) * sizeof(float);
}

template <int BY>
static void launch_by(const Batch &b, const Stage &st, int S, RegArgs a, size_t lds, hipStream_t strm) {
    switch (S) {
        case 1: k_tnlm_reg<1, BY><<<st.grid, kBlock, lds, strm>>>(b, st, a); break;
        case 2: k_tnlm_reg<2, BY><<<st.grid, kBlock, lds, strm>>>(b, st, a); break;
        case 3: k_tnlm_reg<3, BY><<<st.grid, kBlock, lds, strm>>>(b, st, a); break;
        default: k_tnlm_reg<4, BY><<<st.grid, kBlock, lds, strm>>>(b, st, a); break;
    }
}

void launch_regularize(const Batch &b, const Stage &st, const RegParams &p, int rows_per_lane,
                       const float *guide, const float *value, const float *g, float *out, int clamp,
                       double *relpart, int *nonfinite, hipStream_t strm) {
    if (st.total == 0) return;
    RegArgs a;
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
    const size_t lds = reg_lds_bytes(p, rows_per_lane, value == guide);
    if (rows_per_lane == 4) launch_by<4>(b, st, p.patch / 2, a, lds, strm);
    else launch_by<8>(b, st, p.patch / 2, a, lds, strm);
}


// ---------------------------------------------------------------------------
// Symmetric reuse (§2.3): the distance between the patch of x in phase i and
// the patch of y in phase i+1 is also the distance between the patch of y in
// phase i+1 and the patch of x in phase i, so the unnormalised weight
// exp(-D/h^2) of Eq. 8 serves both directions. One block takes one tile T of
// one unordered pair (i, i+1) and every offset of the window:
//   * forward (phase i, pixel x in T, neighbour i+1): sums over the window of
//     w * value_{i+1}(y) and of w, in registers as in the kernel above;
//   * reverse (phase i+1, pixel y = x + delta, neighbour i): the same w times
//     value_i(x), added into an LDS region covering T grown by the window
//     radius; the pixels of that region near its rim also receive terms from
//     the neighbouring tiles, so the block writes the region's sums out and a
//     second kernel adds the (at most four) tiles' sums of each pixel. The
//     sums go to image-shaped planes, one per residue class (ty mod my, tx mod
//     mx) of the tile's position, with my, mx the number of tiles whose
//     regions can hold a pixel along y and x: regions of one class never
//     overlap, every write and every read streams along image rows.
// One exponential and one distance per pair of directions, against two of
// each when every phase computes both neighbours itself. The weights are not
// shifted by the per-pixel minimum, which no single pass can know for the
// reverse direction: exp2(D * nk) <= 1 cannot overflow, and where a pixel's
// weight sum falls below 2^-60 (a best match more than ~40 h^2 away, where
// terms below 2^-126 would be lost) the second kernel recomputes that
// direction of that pixel exactly, with the running minimum.
//
// Waves split the window's offsets in four row-major quarters; each wave owns
// its own reverse region (no two lanes of one wave instruction meet the same
// y, and no two waves share a region), so every sum is taken in a fixed
// order. LDS float atomics cost about eight times a read and a write here,
// so the sums are plain read-add-writes. A region holds sum w v and sum w in
// planes of alternate columns (the 16 lanes of a band touch 16 consecutive
// words) with a row stride that puts bands 0, 1 (and 2, 3) of a wave on
// opposite halves of the 32 banks.

constexpr int kSymBY = 4;   // output rows per lane of the symmetric kernel

struct SymArgs {
    int R, rwh;          // window radius; row stride of one column-parity plane of a reverse region
    float nk;            // -log2(e) / h^2
    const float *guide, *value;
    float2 *fwd;         // [image elements]: forward (sum w v, sum w) of phase i toward i+1
    float2 *part;        // [my * mx][image elements]: reverse (sum w v, sum w) of the tiles' regions
    size_t nimg;         // image elements of the batch (stride of a plane)
    int my, mx;          // region-class counts along y and x
};

template <int S, int kBY>
__global__ __launch_bounds__(kBlock) void k_tnlm_sym(Batch bt, Stage st, SymArgs a) {
#pragma clang fp contract(off)
    extern __shared__ float lds[];
    constexpr int TW = 32 - 2 * S, TH = 4 * kBY, NR = kBY + 2 * S;
    const int R = a.R, W = 2 * R + 1, WW = W * W;
    const int TCW = 32 + 2 * R, TRH = TH + 2 * S + 2 * R, TS = TCW * TRH;
    const int RW = TW + 2 * R, RH = TH + 2 * R;
    const int rwh = a.rwh, pl = RH * rwh;   // pairs in one parity plane
    const bool same = a.value == a.guide;
    float *tg = lds, *tv = same ? lds : lds + TS;
    float *rev = lds + (same ? 1 : 2) * TS;
    __shared__ int sh_item;
    WorkIter it = work_begin(st);
    int gb;
    while (work_next(st, it, gb, &sh_item)) {
        const int sidx = find_slice(st.pre, bt.ns, gb);
        if (bt.skip && bt.skip[sidx]) continue;
        const SliceDesc sd = bt.sl[sidx];
        const int L = sd.L, N = sd.N;
        const int ntx = (L + TW - 1) / TW, nty = (L + TH - 1) / TH;
        const int lb = gb - st.pre[sidx];
        const int tile_local = lb % (ntx * nty);
        const int i = lb / (ntx * nty), j = (i + 1) % N;
        const int x0 = (tile_local % ntx) * TW, y0 = (tile_local / ntx) * TH;
        const size_t plane = (size_t)L * L;
        const float *guide = a.guide + sd.img0, *value = a.value + sd.img0;

        __syncthreads();   // LDS reuse across work items
        const int col0 = x0 - S - R, row0 = y0 - S - R;
        for (int e = threadIdx.x; e < TS; e += kBlock) {
            const int tr = e / TCW, tc = e - tr * TCW;
            const int gr = min(max(row0 + tr, 0), L - 1), gc = min(max(col0 + tc, 0), L - 1);
            const size_t off = (size_t)gr * L + gc;
            tg[e] = guide[j * plane + off];
            if (!same) tv[e] = value[j * plane + off];
        }
        for (int e = threadIdx.x; e < 16 * pl; e += kBlock) rev[e] = 0.0f;

        // the wave index as a wave-uniform value: the offset loop's bounds and
        // the offsets' address parts then live in scalar registers
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
        const int l16 = lane & 15, band = lane >> 4;
        const int xa = x0 - S + 2 * l16;
        const int zbase = y0 + band * kBY - S;
        const int yb = y0 + band * kBY;
        float gia[NR], gib[NR], via[kBY], vib[kBY];
        {
            const float *gi = guide + (size_t)i * plane, *vi = value + (size_t)i * plane;
            const int ca = min(max(xa, 0), L - 1), cb = min(max(xa + 1, 0), L - 1);
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                const int zr = min(max(zbase + k, 0), L - 1);
                gia[k] = gi[(size_t)zr * L + ca];
                gib[k] = gi[(size_t)zr * L + cb];
            }
#pragma unroll
            for (int o = 0; o < kBY; ++o) {
                const int zr = min(yb + o, L - 1);
                via[o] = vi[(size_t)zr * L + ca];
                vib[o] = vi[(size_t)zr * L + cb];
            }
        }
        const bool va = lane_valid_a<S>(l16) && xa >= x0 && xa < x0 + TW && xa < L;
        const bool vb = lane_valid_b<S>(l16) && xa + 1 >= x0 && xa + 1 < x0 + TW && xa + 1 < L;
        float numa[kBY], dena[kBY], numb[kBY], denb[kBY];
#pragma unroll
        for (int o = 0; o < kBY; ++o) numa[o] = dena[o] = numb[o] = denb[o] = 0.0f;
        __syncthreads();

        const int ta = 2 * l16 + R, trb = band * kBY + R;
        const float nk = a.nk;
        // per-lane bases; each offset adds a wave-uniform part
        const float *tgl = tg + trb * TCW + ta;                      // guide tile at (row, column) of x
        const float *tvl = tv + (band * kBY + S + R) * TCW + ta;     // value tile at x's first output row
        float *rwl = rev + wave * 4 * pl + (band * kBY + R) * rwh + l16;   // reverse region, x's first row
        // offsets in column-major order (dy fastest): along a column run a
        // lane's targets y move down one row per offset, so the reverse sums
        // of its BY rows are carried in registers and a row goes to LDS once
        // it has left the lane's window
        const int k0 = wave * WW / 4, k1 = (wave + 1) * WW / 4;
        int dx = k0 / W - R, dy = k0 % W - R;
        float san[kBY], sad[kBY], sbn[kBY], sbd[kBY];   // carried reverse sums, rows j + dy of columns a, b
#pragma unroll
        for (int j = 0; j < kBY; ++j) san[j] = sad[j] = sbn[j] = sbd[j] = 0.0f;
        for (int k = k0; k < k1; ++k) {
            // the neighbour's values at y (in bounds for every lane): read
            // first, so the distance arithmetic hides their latency
            const float *vp = tvl + dy * TCW + dx;
            float vya[kBY], vyb[kBY];
#pragma unroll
            for (int o = 0; o < kBY; ++o) {
                vya[o] = vp[o * TCW];
                vyb[o] = vp[o * TCW + 1];
            }
            // squared differences of the lane's two columns over its BY + 2S
            // rows; summed down the patch rows first (per column, in
            // registers), then across the patch columns (DPP) for the BY
            // output rows only
            float ea[NR], eb[NR];
            const float *rowp = tgl + dy * TCW + dx;
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const float da = gia[q] - rowp[q * TCW];
                const float db = gib[q] - rowp[q * TCW + 1];
                ea[q] = da * da;
                eb[q] = db * db;
            }
            const bool ca = va && (unsigned)(xa + dx) < (unsigned)L;
            const bool cb = vb && (unsigned)(xa + 1 + dx) < (unsigned)L;
            // reverse region column of y = x + delta: 2 l16 + c0 for column a,
            // the next one (other parity plane) for b; c0 is wave-uniform
            const int c0 = dx + R - S;
            const int par = c0 & 1;
            float *ra = rwl + par * pl + (c0 >> 1) + dy * rwh;
            float *rb = rwl + (par ^ 1) * pl + ((c0 + 1) >> 1) + dy * rwh;
            float p2a[NR - 1], p2b[NR - 1];
#pragma unroll
            for (int q = 0; q + 1 < NR; ++q) {
                p2a[q] = ea[q] + ea[q + 1];
                p2b[q] = eb[q] + eb[q + 1];
            }
            float wa[kBY], wva[kBY], wb[kBY], wvb[kBY];   // reverse terms, 0 for pairs outside the image
#pragma unroll
            for (int o = 0; o < kBY; ++o) {
                float Va = ea[o + 2 * S], Vb = eb[o + 2 * S];
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    Va += p2a[o + 2 * q];
                    Vb += p2b[o + 2 * q];
                }
                float Da, Db;
                hsum<S>(Va, Vb, Va + Vb, Da, Db);
                // Both ends inside the image (y's row here, x's row too: rows of
                // the last tile row past the image must not reach y's sums); a
                // pair with an end outside takes an infinite distance, so its
                // weight is exactly 0 and every sum below gains +0 (the staged
                // values are finite): no branches.
                const bool rv = (unsigned)(yb + o + dy) < (unsigned)L && yb + o < L;
                wa[o] = __builtin_amdgcn_exp2f((rv && ca ? Da : INFINITY) * nk);
                wb[o] = __builtin_amdgcn_exp2f((rv && cb ? Db : INFINITY) * nk);
                numa[o] = fmaf(wa[o], vya[o], numa[o]);
                dena[o] += wa[o];
                wva[o] = wa[o] * via[o];
                numb[o] = fmaf(wb[o], vyb[o], numb[o]);
                denb[o] += wb[o];
                wvb[o] = wb[o] * vib[o];
            }
            // reverse sums: carried rows gain this offset's terms; row 0 of the
            // window (y row dy) is final for this column run and goes to LDS
            // (every row of a valid column lies inside the region; adding 0
            // leaves a sum unchanged); at the run's end all rows go
#pragma unroll
            for (int j = 0; j < kBY; ++j) {
                san[j] += wva[j];
                sad[j] += wa[j];
                sbn[j] += wvb[j];
                sbd[j] += wb[j];
            }
            const bool run_end = dy == R || k + 1 == k1;   // wave-uniform
            const int nflush = run_end ? kBY : 1;
            if (va) {
                float n[kBY], d[kBY];
#pragma unroll
                for (int j = 0; j < kBY; ++j)
                    if (j < nflush) {
                        n[j] = ra[j * rwh];
                        d[j] = ra[j * rwh + 2 * pl];
                    }
#pragma unroll
                for (int j = 0; j < kBY; ++j)
                    if (j < nflush) {
                        ra[j * rwh] = n[j] + san[j];
                        ra[j * rwh + 2 * pl] = d[j] + sad[j];
                    }
            }
            if (vb) {
                float n[kBY], d[kBY];
#pragma unroll
                for (int j = 0; j < kBY; ++j)
                    if (j < nflush) {
                        n[j] = rb[j * rwh];
                        d[j] = rb[j * rwh + 2 * pl];
                    }
#pragma unroll
                for (int j = 0; j < kBY; ++j)
                    if (j < nflush) {
                        rb[j * rwh] = n[j] + sbn[j];
                        rb[j * rwh + 2 * pl] = d[j] + sbd[j];
                    }
            }
            // shift the window down one row (a new run starts empty)
#pragma unroll
            for (int j = 0; j < kBY; ++j) {
                const bool keep = !run_end && j + 1 < kBY;
                san[j] = keep ? san[j + 1 < kBY ? j + 1 : j] : 0.0f;
                sad[j] = keep ? sad[j + 1 < kBY ? j + 1 : j] : 0.0f;
                sbn[j] = keep ? sbn[j + 1 < kBY ? j + 1 : j] : 0.0f;
                sbd[j] = keep ? sbd[j + 1 < kBY ? j + 1 : j] : 0.0f;
            }
            // Within one offset the lanes' and rows' targets y = x + delta are
            // all different, so the read-add-writes above need no atomics; a
            // later offset may hit a y another lane wrote here, so no LDS
            // access may move across this point (a wave's LDS operations
            // complete in issue order).
            __asm__ volatile("" ::: "memory");
            if (++dy > R) {
                dy = -R;
                ++dx;
            }
        }

        // ---- reverse: the four waves' regions, added in wave order, into the
        // plane of this tile's class at phase j's elements (inside the image)
        __syncthreads();
        {
            const int ty = y0 / TH, tx = x0 / TW;
            float2 *pt = a.part + (size_t)((ty % a.my) * a.mx + tx % a.mx) * a.nimg + sd.img0 + (size_t)j * plane;
            for (int e = threadIdx.x; e < RH * RW; e += kBlock) {
                const int r = e / RW, c = e - r * RW;
                const int Y = y0 - R + r, X = x0 - R + c;
                if ((unsigned)Y >= (unsigned)L || (unsigned)X >= (unsigned)L) continue;
                const int o = (c & 1) * pl + r * rwh + (c >> 1);
                float n = rev[o], d = rev[o + 2 * pl];
#pragma unroll
                for (int w = 1; w < 4; ++w) {
                    n += rev[w * 4 * pl + o];
                    d += rev[w * 4 * pl + o + 2 * pl];
                }
                pt[(size_t)Y * L + X] = make_float2(n, d);
            }
        }
        // ---- forward: waves 1..3 park their sums in the (now free) region space, wave 0 adds
        __syncthreads();
        float *mg = rev;   // [3][4 * kBY][64]: lane-consecutive words
        if (wave > 0) {
            float *p = mg + (size_t)(wave - 1) * 4 * kBY * 64 + lane;
#pragma unroll
            for (int o = 0; o < kBY; ++o) {
                p[(4 * o + 0) * 64] = numa[o]; p[(4 * o + 1) * 64] = dena[o];
                p[(4 * o + 2) * 64] = numb[o]; p[(4 * o + 3) * 64] = denb[o];
            }
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int w = 0; w < 3; ++w) {
                const float *p = mg + (size_t)w * 4 * kBY * 64 + lane;
#pragma unroll
                for (int o = 0; o < kBY; ++o) {
                    numa[o] += p[(4 * o + 0) * 64]; dena[o] += p[(4 * o + 1) * 64];
                    numb[o] += p[(4 * o + 2) * 64]; denb[o] += p[(4 * o + 3) * 64];
                }
            }
            float2 *fo = a.fwd + sd.img0 + (size_t)i * plane;
#pragma unroll
            for (int o = 0; o < kBY; ++o) {
                if (yb + o >= L) continue;
                if (va) fo[(size_t)(yb + o) * L + xa] = make_float2(numa[o], dena[o]);
                if (vb) fo[(size_t)(yb + o) * L + xa + 1] = make_float2(numb[o], denb[o]);
            }
        }
    }
    work_end(st);
}

// One direction of one pixel exactly as Eq. 8 states it (direct patch sums,
// running minimum): the fallback where the unshifted weights underflow.
__device__ __noinline__ float exact_side(const float *__restrict__ gi, const float *__restrict__ gj,
                            const float *__restrict__ vj, int L, int S, int R, float nk, int r, int c) {
    float Dm = INFINITY, num = 0.0f, den = 0.0f;
    for (int dy = -R; dy <= R; ++dy) {
        const int r2 = r + dy;
        if (r2 < 0 || r2 >= L) continue;
        for (int dx = -R; dx <= R; ++dx) {
            const int c2 = c + dx;
            if (c2 < 0 || c2 >= L) continue;
            float D = 0.0f;
            for (int py = -S; py <= S; ++py) {
                const int ra = min(max(r + py, 0), L - 1), rb = min(max(r2 + py, 0), L - 1);
                for (int px = -S; px <= S; ++px) {
                    const int ca = min(max(c + px, 0), L - 1), cb = min(max(c2 + px, 0), L - 1);
                    const float d = gi[(size_t)ra * L + ca] - gj[(size_t)rb * L + cb];
                    D = fmaf(d, d, D);
                }
            }
            online_add(D, vj[(size_t)r2 * L + c2], nk, Dm, num, den);
        }
    }
    return num / den;
}

struct SymFinishArgs {
    int R;
    float nk, cs, cn;
    const float *guide, *value, *g;
    const float2 *fwd;
    const float2 *part;
    size_t nimg;
    int my, mx;
    float *out;
    int clamp;
    double *relpart;
    int *nonfinite;
};

// Eq. 7 from the two directions of each pixel: the forward sums of the pair
// (i, i+1) and the reverse sums of the pair (i-1, i) from every tile whose
// region holds the pixel (tile rows, then columns, ascending).
template <int S, int kBY>
__global__ __launch_bounds__(kBlock) void k_tnlm_sym_finish(Batch bt, Stage st, SymFinishArgs a) {
#pragma clang fp contract(off)
    __shared__ double shred[kBlock];
    __shared__ int sh_item;
    const float tiny = 0x1p-60f;
    constexpr int TW = 32 - 2 * S, TH = 4 * kBY;   // compile-time: the index divisions become multiplies
    const int R = a.R;
    const int RW = TW + 2 * R, RH = TH + 2 * R;
    WorkIter it = work_begin(st);
    int gb;
    while (work_next(st, it, gb, &sh_item)) {
        const int sidx = find_slice(st.pre, bt.ns, gb);
        if (bt.skip && bt.skip[sidx]) continue;
        const SliceDesc sd = bt.sl[sidx];
        const int L = sd.L, N = sd.N;
        const int ntx = (L + TW - 1) / TW, nty = (L + TH - 1) / TH, nt = ntx * nty;
        const int lb = gb - st.pre[sidx];
        const int tile_local = lb % nt, i = lb / nt;
        const int x0 = (tile_local % ntx) * TW, y0 = (tile_local / ntx) * TH;
        const int ip = (i - 1 + N) % N, in = (i + 1) % N;
        const size_t plane = (size_t)L * L;
        const float *gs = a.guide + sd.img0, *vs = a.value + sd.img0;
        const float *gi = a.g + sd.img0 + (size_t)i * plane;
        float *oi = a.out + sd.img0 + (size_t)i * plane;
        const float2 *fw = a.fwd + sd.img0 + (size_t)i * plane;
        const float2 *pp = a.part + sd.img0 + (size_t)i * plane;   // phase i's elements of plane 0
        double dd = 0.0, nn = 0.0;
        bool bad = false;
        for (int e = threadIdx.x; e < TW * TH; e += kBlock) {
            const int r = y0 + e / TW, c = x0 + e % TW;
            if (r >= L || c >= L) continue;
            const size_t px = (size_t)r * L + c;
            // tiles t whose region [t*T - R, t*T + T + R) holds the row / column:
            // ceil((r - R - T + 1) / T) <= t <= floor((r + R) / T), the lower
            // bound's numerator made positive by 64 T (R < 64 <= 64 T)
            const int tylo = max(0, (r - R + 64 * TH) / TH - 64);
            const int txlo = max(0, (c - R + 64 * TW) / TW - 64);
            const int tyhi = min(nty - 1, (r + R) / TH), txhi = min(ntx - 1, (c + R) / TW);
            float nr = 0.0f, dr = 0.0f;
            for (int ty = tylo; ty <= tyhi; ++ty)
                for (int tx = txlo; tx <= txhi; ++tx) {
                    const float2 v = pp[(size_t)((ty % a.my) * a.mx + tx % a.mx) * a.nimg + px];
                    nr += v.x;
                    dr += v.y;
                }
            const float2 F = fw[px];
            const float Ar = dr >= tiny ? nr / dr
                                        : exact_side(gs + (size_t)i * plane, gs + (size_t)ip * plane,
                                                     vs + (size_t)ip * plane, L, S, R, a.nk, r, c);
            const float Af = F.y >= tiny ? F.x / F.y
                                         : exact_side(gs + (size_t)i * plane, gs + (size_t)in * plane,
                                                      vs + (size_t)in * plane, L, S, R, a.nk, r, c);
            float u = fmaf(a.cn, Ar + Af, a.cs * gi[px]);
            if (a.clamp) u = fmaxf(u, 0.0f);
            if (a.relpart) {
                const double df = (double)u - (double)oi[px];
                dd = fma(df, df, dd);
                nn = fma((double)u, (double)u, nn);
            }
            bad |= !isfinite(u);
            oi[px] = u;
        }
        if (bad && a.nonfinite) a.nonfinite[sidx] = 1;
        if (a.relpart) {
            dd = block_sum_256(dd, shred);
            nn = block_sum_256(nn, shred);
            if (threadIdx.x == 0) {
                const long long blk = (long long)sd.rp0 + lb;
                a.relpart[2 * blk] = dd;
                a.relpart[2 * blk + 1] = nn;
            }
        }
    }
    work_end(st);
}

// Row stride of one column-parity plane of a reverse region: at least half
// the region's width, with 4 * stride = 16 (mod 32) so that bands 0, 1 (2, 3)
// of a wave fall on opposite bank halves; the plain half width where that
// would not fit. Also the LDS bytes of a block.
static int sym_rwh(int patch, int window, bool same, size_t *lds_bytes) {
    const int S = patch / 2, R = window / 2;
    const int RW = 32 - 2 * S + 2 * R, RH = 4 * kSymBY + 2 * R;
    const size_t ts = (size_t)(32 + 2 * R) * (4 * kSymBY + 2 * S + 2 * R) * (same ? 1 : 2);
    int rwh = (RW + 1) / 2;
    while (rwh % 8 != 4) ++rwh;
    if ((ts + 16 * (size_t)RH * rwh) * sizeof(float) > 65536) rwh = (RW + 1) / 2;
    const size_t need = std::max(ts + 16 * (size_t)RH * rwh, ts + (size_t)3 * 64 * 4 * kSymBY) * sizeof(float);
    if (lds_bytes) *lds_bytes = need;
    return rwh;
}

bool reg_sym_supported(int patch, int window) {
    if (!reg_supported(patch, window)) return false;
    size_t a = 0, b = 0;
    sym_rwh(patch, window, true, &a);
    sym_rwh(patch, window, false, &b);
    return std::max(a, b) <= 65536;
}

// Region classes along y and x: the number of tiles whose regions (the tile
// grown by R) can hold one pixel.
static void sym_classes(int patch, int window, int &my, int &mx) {
    const int S = patch / 2, R = window / 2, TW = 32 - 2 * S, TH = 4 * kSymBY;
    my = (TH + 2 * R + TH - 1) / TH;
    mx = (TW + 2 * R + TW - 1) / TW;
}

int reg_sym_planes(int patch, int window) {
    int my, mx;
    sym_classes(patch, window, my, mx);
    return my * mx;
}

int reg_sym_rows_per_lane() { return kSymBY; }

void launch_regularize_sym(const Batch &b, const Stage &st, const RegParams &p, const float *guide,
                           const float *value, const float *g, float *out, int clamp, double *relpart,
                           int *nonfinite, float2 *fwd, float2 *part, size_t nimg, hipStream_t strm) {
    if (st.total == 0) return;
    size_t lds = 0;
    SymArgs a;
    a.R = p.window / 2;
    a.rwh = sym_rwh(p.patch, p.window, value == guide, &lds);
    a.nk = (float)(-1.4426950408889634 / ((double)p.h * (double)p.h));
    a.guide = guide;
    a.value = value;
    a.fwd = fwd;
    a.part = part;
    a.nimg = nimg;
    sym_classes(p.patch, p.window, a.my, a.mx);
    switch (p.patch / 2) {
        case 1: k_tnlm_sym<1, kSymBY><<<st.grid, kBlock, lds, strm>>>(b, st, a); break;
        case 2: k_tnlm_sym<2, kSymBY><<<st.grid, kBlock, lds, strm>>>(b, st, a); break;
        case 3: k_tnlm_sym<3, kSymBY><<<st.grid, kBlock, lds, strm>>>(b, st, a); break;
        default: k_tnlm_sym<4, kSymBY><<<st.grid, kBlock, lds, strm>>>(b, st, a); break;
    }
    SymFinishArgs f;
    f.R = p.window / 2;
    f.nk = a.nk;
    f.cs = (float)(1.0 / (1.0 + (double)p.mu_hat));
    f.cn = (float)((double)p.mu_hat / (2.0 * (double)p.mu_hat + 2.0));
    f.guide = guide;
    f.value = value;
    f.g = g;
    f.fwd = fwd;
    f.part = part;
    f.nimg = nimg;
    f.my = a.my;
    f.mx = a.mx;
    f.out = out;
    f.clamp = clamp;
    f.relpart = relpart;
    f.nonfinite = nonfinite;
    // the combining pass streams through its tiles: the fixed per-XCD ranges,
    // without the work counters (one atomic round trip per tile)
    Stage fs = st;
    fs.queue = nullptr;
    switch (p.patch / 2) {
        case 1: k_tnlm_sym_finish<1, kSymBY><<<st.grid, kBlock, 0, strm>>>(b, fs, f); break;
        case 2: k_tnlm_sym_finish<2, kSymBY><<<st.grid, kBlock, 0, strm>>>(b, fs, f); break;
        case 3: k_tnlm_sym_finish<3, kSymBY><<<st.grid, kBlock, 0, strm>>>(b, fs, f); break;
        default: k_tnlm_sym_finish<4, kSymBY><<<st.grid, kBlock, 0, strm>>>(b, fs, f); break;
    }
}

}  // namespace tnlm
