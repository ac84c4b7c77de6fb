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
#include "devutil.h"
#include "internal.h"

namespace tnlm {

__global__ void k_sqrt(const float *__restrict__ w, float *__restrict__ sw, size_t n) {
    size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; k < n; k += (size_t)gridDim.x * blockDim.x) sw[k] = sqrtf(fmaxf(w[k], 0.0f));
}

void launch_sqrt(const float *w, float *sw, size_t n, hipStream_t st) {
    int nb = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
    k_sqrt<<<nb, kBlock, 0, st>>>(w, sw, n);
}

__global__ void k_copy(const float *__restrict__ a, float *__restrict__ b, size_t n, const int *skip) {
    if (skip_now(skip)) return;
    size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; k < n; k += (size_t)gridDim.x * blockDim.x) b[k] = a[k];
}

void launch_copy(const float *src, float *dst, size_t n, const int *skip, hipStream_t st) {
    int nb = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
    k_copy<<<nb, kBlock, 0, st>>>(src, dst, n, skip);
}

// Step m: a = gamma/||q||^2, u += a s (image part), r -= a q and rw = sw r (sinogram part).
__global__ __launch_bounds__(kBlock) void k_cgls_update(int nimg, int nsino, const double *__restrict__ gpart,
                                                        int nbp, const double *__restrict__ qpart, int npp,
                                                        int *__restrict__ stop, int m, int N,
                                                        float *__restrict__ u, const float *__restrict__ s,
                                                        float *__restrict__ r, const float *__restrict__ q,
                                                        float *__restrict__ rw, const float *__restrict__ sw,
                                                        const int *skip) {
    __shared__ double sh[kBlock];
    if (skip_now(skip)) return;
    const int i = blockIdx.y;
    const double gamma = block_sum_array(gpart + (size_t)i * nbp, nbp, sh);
    const double qq = block_sum_array(qpart + (size_t)i * npp, npp, sh);
    const int stopped_before = m > 0 ? stop[(size_t)m * N + i] : 0;
    const int stopped = stopped_before || !(gamma > 0.0) || !(qq > 0.0);
    if (blockIdx.x == 0 && threadIdx.x == 0) stop[(size_t)(m + 1) * N + i] = stopped;
    if (stopped) return;
    const float a = (float)(gamma / qq);
    const size_t tot = (size_t)nimg + nsino;
    for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < tot; k += (size_t)gridDim.x * kBlock) {
        if (k < (size_t)nimg) {
            const size_t e = (size_t)i * nimg + k;
            u[e] = fmaf(a, s[e], u[e]);
        } else {
            const size_t e = (size_t)i * nsino + (k - nimg);
            const float rv = fmaf(-a, q[e], r[e]);
            r[e] = rv;
            rw[e] = sw[e] * rv;
        }
    }
}

static int vec_blocks(size_t n) { return (int)std::max<size_t>(1, std::min<size_t>((n + 4 * kBlock - 1) / (4 * kBlock), 512)); }

void launch_cgls_update(const DevGeom &g, CglsBufs &b, int m, int gsel, const int *skip, hipStream_t st) {
    const int nimg = g.L * g.L, nsino = g.V * g.B;
    dim3 grid(vec_blocks((size_t)nimg + nsino), g.N);
    k_cgls_update<<<grid, kBlock, 0, st>>>(nimg, nsino, b.gpart[gsel], b.nbp, b.qpart, b.npp, b.stop, m, g.N,
                                           b.u, b.s, b.r, b.q, b.rw, b.sw, skip);
}

// s = t + (gamma_new / gamma_old) s
__global__ __launch_bounds__(kBlock) void k_cgls_direction(int nimg, const double *__restrict__ gold,
                                                           const double *__restrict__ gnew, int nbp,
                                                           const int *__restrict__ stop, int m, int N,
                                                           float *__restrict__ s, const float *__restrict__ t,
                                                           const int *skip) {
    __shared__ double sh[kBlock];
    if (skip_now(skip)) return;
    const int i = blockIdx.y;
    if (stop[(size_t)(m + 1) * N + i]) return;
    const double go = block_sum_array(gold + (size_t)i * nbp, nbp, sh);
    const double gn = block_sum_array(gnew + (size_t)i * nbp, nbp, sh);
    const float bc = (float)(gn / go);
    for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < (size_t)nimg; k += (size_t)gridDim.x * kBlock) {
        const size_t e = (size_t)i * nimg + k;
        s[e] = fmaf(bc, s[e], t[e]);
    }
}

void launch_cgls_direction(const DevGeom &g, CglsBufs &b, int m, int gsel_old, int gsel_new, const int *skip,
                           hipStream_t st) {
    const int nimg = g.L * g.L;
    dim3 grid(vec_blocks(nimg), g.N);
    k_cgls_direction<<<grid, kBlock, 0, st>>>(nimg, b.gpart[gsel_old], b.gpart[gsel_new], b.nbp, b.stop, m, g.N,
                                              b.s, b.t, skip);
}

// Eq. 4 helpers: tmp = w (P f - y); g = f - (1/beta) P^T tmp
__global__ void k_weighted_resid(size_t n, const float *__restrict__ q, const float *__restrict__ y,
                                 const float *__restrict__ w, float *__restrict__ out, const int *skip) {
    if (skip_now(skip)) return;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        out[k] = w[k] * (q[k] - y[k]);
}

void launch_weighted_resid(const DevGeom &g, const float *q, const float *y, const float *w, float *out,
                           const int *skip, hipStream_t st) {
    size_t n = (size_t)g.N * g.V * g.B;
    k_weighted_resid<<<vec_blocks(n), kBlock, 0, st>>>(n, q, y, w, out, skip);
}

__global__ void k_gradient_step(size_t n, const float *__restrict__ f, const float *__restrict__ bp, float inv_beta,
                                float *__restrict__ g, const int *skip) {
    if (skip_now(skip)) return;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        g[k] = fmaf(-inv_beta, bp[k], f[k]);
}

void launch_gradient_step(const DevGeom &g, const float *f, const float *bp, float inv_beta, float *gout,
                          const int *skip, hipStream_t st) {
    size_t n = (size_t)g.N * g.L * g.L;
    k_gradient_step<<<vec_blocks(n), kBlock, 0, st>>>(n, f, bp, inv_beta, gout, skip);
}

// Outer-loop bookkeeping (one block): relative update from the regulariser's
// partials [nblocks][2] = (sum (f_new - f_old)^2, sum f_new^2), history,
// iteration counter, convergence / non-finite stop flag.
__global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ partials, int nblocks, float tol,
                                                     float *__restrict__ hist, int *__restrict__ counter,
                                                     int *__restrict__ done, const int *__restrict__ nonfinite,
                                                     int max_outer, const int *skip) {
    __shared__ double sh[kBlock];
    if (skip_now(skip)) return;
    double dd = 0.0, nn = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += kBlock) {
        dd += partials[2 * k];
        nn += partials[2 * k + 1];
    }
    dd = block_sum_256(dd, sh);
    nn = block_sum_256(nn, sh);
    if (threadIdx.x == 0) {
        const double rel = sqrt(dd) / fmax(sqrt(nn), 1e-30);
        const int k = *counter;
        if (k < max_outer) hist[k] = (float)rel;
        *counter = k + 1;
        if ((tol > 0.0f && rel < (double)tol) || *nonfinite) *done = 1;
    }
}

void launch_finalize(const double *partials, int nblocks, float tol, float *hist, int *counter, int *done,
                     int *nonfinite, int max_outer, const int *skip, hipStream_t st) {
    k_finalize<<<1, kBlock, 0, st>>>(partials, nblocks, tol, hist, counter, done, nonfinite, max_outer, skip);
}

__global__ void k_check_finite(const float *__restrict__ a, size_t n, int *flag) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        if (!isfinite(a[k])) *flag = 1;
}

void launch_check_finite(const float *a, size_t n, int *flag, hipStream_t st) {
    k_check_finite<<<vec_blocks(n), kBlock, 0, st>>>(a, n, flag);
}

}  // namespace tnlm
