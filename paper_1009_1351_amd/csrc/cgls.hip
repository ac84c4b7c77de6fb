// Vector work of the data step (§2.2, CGLS box) and of the outer loop.
//
// CGLS on P_n = S^-1/2 P, y_n = S^-1/2 y (w = S^-1 diagonal, sw = sqrt(w)):
//   init : r = sw (y - P u) ; s = P^T (sw r) ; gamma = ||s||^2
//   step : q = sw P s ; a = gamma / ||q||^2 ; u += a s ; r -= a q
//          t = P^T (sw r) ; gamma' = ||t||^2 ; s = t + (gamma'/gamma) s
// The projector kernels fuse the sw scalings and emit per-block partial sums;
// the kernels here reduce those partials in a fixed order (every block the
// same order, so every block gets the same scalar) and apply the updates.
// A phase whose ||P_n^T r||^2 or ||P_n s||^2 is exactly zero stops: a = 0 from
// then on, u unchanged.
//
// Work items are (slice, phase, chunk) over the batch's slice table; a chunk
// covers a contiguous range of the phase's image (and sinogram) elements.
#include "devutil.h"
#include "internal.h"

namespace tnlm {

constexpr int kMaxVecBlocks = 64;

int vec_blocks(const SliceDesc &s) {
    const long long n = (long long)s.L * s.L + (long long)s.V * s.B;
    return (int)std::max<long long>(1, std::min<long long>((n + 4 * kBlock - 1) / (4 * kBlock), kMaxVecBlocks));
}

struct VecItem {
    int s, i, chunk, nchunk;
};

__device__ __forceinline__ VecItem vec_item(const Stage &st, int ns, int gb, const SliceDesc *sl, SliceDesc &sd) {
    VecItem it;
    it.s = find_slice(st.pre, ns, gb);
    sd = sl[it.s];
    const int lb = gb - st.pre[it.s];
    it.nchunk = (st.pre[it.s + 1] - st.pre[it.s]) / sd.N;
    it.i = lb / it.nchunk;
    it.chunk = lb - it.i * it.nchunk;
    return it;
}

__device__ __forceinline__ void chunk_range(long long n, int chunk, int nchunk, long long &lo, long long &hi) {
    const long long per = (n + nchunk - 1) / nchunk;
    lo = std::min(n, (long long)chunk * per);
    hi = std::min(n, lo + per);
}

// Elements [n0, n1) (indices into arrays that start 16-byte aligned) by the
// block: the aligned middle four at a time (16-byte accesses), the at most
// three elements before and after it one at a time.
template <class V, class S>
__device__ __forceinline__ void vec_range(long long n0, long long n1, V vec4, S one) {
    const long long v0 = std::min(n1, (n0 + 3) & ~3LL);
    const long long v1 = std::max(v0, n1 & ~3LL);
    if ((long long)threadIdx.x < v0 - n0) one(n0 + threadIdx.x);
    if ((long long)threadIdx.x < n1 - v1) one(v1 + threadIdx.x);
    for (long long k = v0 + 4 * (long long)threadIdx.x; k < v1; k += 4 * kBlock) vec4(k);
}

__global__ void k_sqrt(const float *__restrict__ w, float *__restrict__ sw, size_t n) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        sw[k] = sqrtf(fmaxf(w[k], 0.0f));
}

static int flat_blocks(size_t n) { return (int)std::max<size_t>(1, std::min<size_t>((n + kBlock - 1) / kBlock, 4096)); }

void launch_sqrt(const float *w, float *sw, size_t n, hipStream_t st) {
    k_sqrt<<<flat_blocks(n), kBlock, 0, st>>>(w, sw, n);
}

__global__ void k_copy(const float *__restrict__ a, float *__restrict__ b, size_t n) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        b[k] = a[k];
}

void launch_copy(const float *src, float *dst, size_t n, hipStream_t st) {
    k_copy<<<flat_blocks(n), kBlock, 0, st>>>(src, dst, n);
}

// Per-slice copy (image- or sinogram-shaped), skipping stopped slices.
__global__ __launch_bounds__(kBlock) void k_copy_skip(Batch bt, Stage st, int image, const float *__restrict__ a,
                                                      float *__restrict__ b) {
    for (int gb = blockIdx.x, gend = stage_total(st); gb < gend; gb += gridDim.x) {
        SliceDesc sd;
        const VecItem it = vec_item(st, bt.ns, gb, bt.sl, sd);
        if (bt.skip && bt.skip[it.s]) continue;
        const long long n = image ? (long long)sd.L * sd.L : (long long)sd.V * sd.B;
        const long long base = (image ? sd.img0 : sd.sino0) + (long long)it.i * n;
        long long lo, hi;
        chunk_range(n, it.chunk, it.nchunk, lo, hi);
        for (long long k = lo + threadIdx.x; k < hi; k += kBlock) b[base + k] = a[base + k];
    }
}

void launch_copy_skip(const Batch &b, const Stage &st, bool image, const float *src, float *dst, hipStream_t strm) {
    k_copy_skip<<<st.grid, kBlock, 0, strm>>>(b, st, image ? 1 : 0, src, dst);
}

// Step m: a = gamma/||q||^2, u += a s (image part), r -= a q and rw = sw r (sinogram part).
__global__ __launch_bounds__(kBlock) void k_cgls_update(Batch bt, Stage st, CglsBufs cb, int m, int gsel) {
    __shared__ double sh[kBlock];
    for (int gb = blockIdx.x, gend = stage_total(st); gb < gend; gb += gridDim.x) {
        SliceDesc sd;
        const VecItem it = vec_item(st, bt.ns, gb, bt.sl, sd);
        if (bt.skip && bt.skip[it.s]) continue;
        const double gamma = block_sum_array(cb.gpart[gsel] + sd.gp0 + (long long)it.i * sd.nbp, sd.nbp, sh);
        const double qq = block_sum_array(cb.qpart + sd.qp0 + (long long)it.i * sd.npp, sd.npp, sh);
        const int gp = sd.phase0 + it.i;
        const int stopped_before = m > 0 ? cb.stop[(long long)m * cb.nphase + gp] : 0;
        const int stopped = stopped_before || !(gamma > 0.0) || !(qq > 0.0);
        if (it.chunk == 0 && threadIdx.x == 0) cb.stop[(long long)(m + 1) * cb.nphase + gp] = stopped;
        if (stopped) continue;
        const float a = (float)(gamma / qq);
        const long long nimg = (long long)sd.L * sd.L, nsino = (long long)sd.V * sd.B;
        long long lo, hi;
        chunk_range(nimg + nsino, it.chunk, it.nchunk, lo, hi);
        const long long ib = sd.img0 + (long long)it.i * nimg, sbase = sd.sino0 + (long long)it.i * nsino;
        float *__restrict__ u = cb.u;
        const float *__restrict__ sv = cb.s;
        if (lo < nimg)
            vec_range(
                ib + lo, ib + std::min(hi, nimg),
                [&](long long k) {
                    const float4 s4 = *reinterpret_cast<const float4 *>(sv + k);
                    float4 u4 = *reinterpret_cast<const float4 *>(u + k);
                    u4.x = fmaf(a, s4.x, u4.x);
                    u4.y = fmaf(a, s4.y, u4.y);
                    u4.z = fmaf(a, s4.z, u4.z);
                    u4.w = fmaf(a, s4.w, u4.w);
                    *reinterpret_cast<float4 *>(u + k) = u4;
                },
                [&](long long k) { u[k] = fmaf(a, sv[k], u[k]); });
        if (hi > nimg) {
            float *__restrict__ r = cb.r, *__restrict__ rw = cb.rw;
            const float *__restrict__ q = cb.q, *__restrict__ sw = cb.sw;
            vec_range(
                sbase + std::max(lo, nimg) - nimg, sbase + hi - nimg,
                [&](long long e) {
                    const float4 q4 = *reinterpret_cast<const float4 *>(q + e);
                    const float4 w4 = *reinterpret_cast<const float4 *>(sw + e);
                    float4 r4 = *reinterpret_cast<const float4 *>(r + e);
                    r4.x = fmaf(-a, q4.x, r4.x);
                    r4.y = fmaf(-a, q4.y, r4.y);
                    r4.z = fmaf(-a, q4.z, r4.z);
                    r4.w = fmaf(-a, q4.w, r4.w);
                    *reinterpret_cast<float4 *>(r + e) = r4;
                    *reinterpret_cast<float4 *>(rw + e) = make_float4(w4.x * r4.x, w4.y * r4.y, w4.z * r4.z, w4.w * r4.w);
                },
                [&](long long e) {
                    const float rv = fmaf(-a, q[e], r[e]);
                    r[e] = rv;
                    rw[e] = sw[e] * rv;
                });
        }
    }
}

void launch_cgls_update(const Batch &b, const Stage &st, CglsBufs &cb, int m, int gsel, hipStream_t strm) {
    k_cgls_update<<<st.grid, kBlock, 0, strm>>>(b, st, cb, m, gsel);
}

// s = t + (gamma_new / gamma_old) s
__global__ __launch_bounds__(kBlock) void k_cgls_direction(Batch bt, Stage st, CglsBufs cb, int m, int gold,
                                                           int gnew) {
    __shared__ double sh[kBlock];
    for (int gb = blockIdx.x, gend = stage_total(st); gb < gend; gb += gridDim.x) {
        SliceDesc sd;
        const VecItem it = vec_item(st, bt.ns, gb, bt.sl, sd);
        if (bt.skip && bt.skip[it.s]) continue;
        if (cb.stop[(long long)(m + 1) * cb.nphase + sd.phase0 + it.i]) continue;
        const double go = block_sum_array(cb.gpart[gold] + sd.gp0 + (long long)it.i * sd.nbp, sd.nbp, sh);
        const double gn = block_sum_array(cb.gpart[gnew] + sd.gp0 + (long long)it.i * sd.nbp, sd.nbp, sh);
        const float bc = (float)(gn / go);
        const long long nimg = (long long)sd.L * sd.L;
        long long lo, hi;
        chunk_range(nimg, it.chunk, it.nchunk, lo, hi);
        const long long ib = sd.img0 + (long long)it.i * nimg;
        float *__restrict__ sv = cb.s;
        const float *__restrict__ tv = cb.t;
        vec_range(
            ib + lo, ib + hi,
            [&](long long k) {
                const float4 t4 = *reinterpret_cast<const float4 *>(tv + k);
                float4 s4 = *reinterpret_cast<const float4 *>(sv + k);
                s4.x = fmaf(bc, s4.x, t4.x);
                s4.y = fmaf(bc, s4.y, t4.y);
                s4.z = fmaf(bc, s4.z, t4.z);
                s4.w = fmaf(bc, s4.w, t4.w);
                *reinterpret_cast<float4 *>(sv + k) = s4;
            },
            [&](long long k) { sv[k] = fmaf(bc, sv[k], tv[k]); });
    }
}

void launch_cgls_direction(const Batch &b, const Stage &st, CglsBufs &cb, int m, int gold, int gnew,
                           hipStream_t strm) {
    k_cgls_direction<<<st.grid, kBlock, 0, strm>>>(b, st, cb, m, gold, gnew);
}

// Eq. 4 helpers: tmp = w (P f - y); g = f - (1/beta) P^T tmp
__global__ __launch_bounds__(kBlock) void k_weighted_resid(Batch bt, Stage st, const float *__restrict__ q,
                                                           const float *__restrict__ y, const float *__restrict__ w,
                                                           float *__restrict__ out) {
    for (int gb = blockIdx.x, gend = stage_total(st); gb < gend; gb += gridDim.x) {
        SliceDesc sd;
        const VecItem it = vec_item(st, bt.ns, gb, bt.sl, sd);
        if (bt.skip && bt.skip[it.s]) continue;
        const long long n = (long long)sd.V * sd.B, base = sd.sino0 + (long long)it.i * n;
        long long lo, hi;
        chunk_range(n, it.chunk, it.nchunk, lo, hi);
        for (long long k = lo + threadIdx.x; k < hi; k += kBlock) out[base + k] = w[base + k] * (q[base + k] - y[base + k]);
    }
}

void launch_weighted_resid(const Batch &b, const Stage &st, const float *q, const float *y, const float *w,
                           float *out, hipStream_t strm) {
    k_weighted_resid<<<st.grid, kBlock, 0, strm>>>(b, st, q, y, w, out);
}

__global__ __launch_bounds__(kBlock) void k_gradient_step(Batch bt, Stage st, const float *__restrict__ f,
                                                          const float *__restrict__ bp, float inv_beta,
                                                          float *__restrict__ g) {
    for (int gb = blockIdx.x, gend = stage_total(st); gb < gend; gb += gridDim.x) {
        SliceDesc sd;
        const VecItem it = vec_item(st, bt.ns, gb, bt.sl, sd);
        if (bt.skip && bt.skip[it.s]) continue;
        const long long n = (long long)sd.L * sd.L, base = sd.img0 + (long long)it.i * n;
        long long lo, hi;
        chunk_range(n, it.chunk, it.nchunk, lo, hi);
        for (long long k = lo + threadIdx.x; k < hi; k += kBlock) g[base + k] = fmaf(-inv_beta, bp[base + k], f[base + k]);
    }
}

void launch_gradient_step(const Batch &b, const Stage &st, const float *f, const float *bp, float inv_beta,
                          float *gout, hipStream_t strm) {
    k_gradient_step<<<st.grid, kBlock, 0, strm>>>(b, st, f, bp, inv_beta, gout);
}

// Outer-loop bookkeeping, one block per slice: relative update from the
// regulariser's partials (sum (f_new - f_old)^2, sum f_new^2), history,
// iteration counter, convergence / non-finite stop flag.
__global__ __launch_bounds__(kBlock) void k_finalize(Batch bt, const double *__restrict__ partials, float tol,
                                                     float *__restrict__ hist, int *__restrict__ counter,
                                                     int *__restrict__ done, const int *__restrict__ nonfinite,
                                                     int max_outer) {
    __shared__ double sh[kBlock];
    const int s = blockIdx.x;
    if (bt.skip && bt.skip[s]) return;
    const SliceDesc sd = bt.sl[s];
    double dd = 0.0, nn = 0.0;
    for (int k = threadIdx.x; k < sd.nrb; k += kBlock) {
        dd += partials[2 * ((long long)sd.rp0 + k)];
        nn += partials[2 * ((long long)sd.rp0 + k) + 1];
    }
    dd = block_sum_256(dd, sh);
    nn = block_sum_256(nn, sh);
    if (threadIdx.x == 0) {
        const double rel = sqrt(dd) / fmax(sqrt(nn), 1e-30);
        const int k = counter[s];
        if (k < max_outer) hist[(long long)s * max_outer + k] = (float)rel;
        counter[s] = k + 1;
        if ((tol > 0.0f && rel < (double)tol) || nonfinite[s]) done[s] = 1;
    }
}

void launch_finalize(const Batch &b, const double *relpart, float tol, float *hist, int *counter, int *done,
                     const int *nonfinite, int max_outer, hipStream_t strm) {
    k_finalize<<<b.ns, kBlock, 0, strm>>>(b, relpart, tol, hist, counter, done, nonfinite, max_outer);
}

__global__ void k_check_finite(const float *__restrict__ a, size_t n, int *flag) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        if (!isfinite(a[k])) *flag = 1;
}

void launch_check_finite(const float *a, size_t n, int *flag, hipStream_t st) {
    k_check_finite<<<flat_blocks(n), kBlock, 0, st>>>(a, n, flag);
}

// sum of w (q - y)^2: per-block partials (FP64), at most 1024 blocks
__global__ __launch_bounds__(kBlock) void k_wsq_sum(const float *__restrict__ q, const float *__restrict__ y,
                                                    const float *__restrict__ w, size_t n, double *__restrict__ part) {
    __shared__ double sh[kBlock];
    double s = 0.0;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        const double d = (double)q[k] - (double)y[k];
        s += (double)w[k] * d * d;
    }
    s = block_sum_256(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

int launch_wsq_sum(const float *q, const float *y, const float *w, size_t n, double *part, hipStream_t st) {
    const int nb = std::min(flat_blocks(n), 1024);
    k_wsq_sum<<<nb, kBlock, 0, st>>>(q, y, w, n, part);
    return nb;
}

// Partial sums of (a - b)^2 and a^2 (double) and a count of non-finite
// entries of a or b, for the relative change ||a - b|| / ||a||.
__global__ __launch_bounds__(kBlock) void k_diff_sq(const float *__restrict__ a, const float *__restrict__ b,
                                                    size_t n, double *__restrict__ part, int *__restrict__ bad) {
    __shared__ double sh[kBlock];
    double d2 = 0.0, a2 = 0.0;
    int nb = 0;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        const float x = a[k], z = b[k];
        if (!isfinite(x) || !isfinite(z)) {
            ++nb;
            continue;
        }
        const double d = (double)x - (double)z;
        d2 += d * d;
        a2 += (double)x * (double)x;
    }
    d2 = block_sum_256(d2, sh);
    a2 = block_sum_256(a2, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = d2;
        part[2 * blockIdx.x + 1] = a2;
    }
    if (nb) atomicAdd(bad, nb);
}

int launch_diff_sq(const float *a, const float *b, size_t n, double *part, int *bad, hipStream_t st) {
    const int nb = std::min(flat_blocks(n), 512);
    k_diff_sq<<<nb, kBlock, 0, st>>>(a, b, n, part, bad);
    return nb;
}

__global__ void k_fill_int(int *a, int n, int v) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) a[k] = v;
}

void launch_fill_int(int *a, int n, int v, hipStream_t st) {
    if (n > 0) k_fill_int<<<std::max(1, std::min((n + kBlock - 1) / kBlock, 1024)), kBlock, 0, st>>>(a, n, v);
}

}  // namespace tnlm
