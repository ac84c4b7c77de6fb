// Siddon forward projector P and its exact transpose P^T for the fan-beam arc
// geometry of §3 (P_i of Eq. 1; P^T of Eq. 4 and the CGLS box).
//
// Both kernels evaluate a ray's parametric crossing with grid line k through
// one shared formula, T(k) = fma(k, A, B), from per-ray constants (A, B)
// built once on the host in double precision. The segment of a ray inside
// pixel (r, c) is the clip
//     l = min(T_x(hi c), T_y(hi r)) - max(T_x(lo c), T_y(lo r)),
// which the forward kernel meets while walking the ray and the transpose
// kernel evaluates for each candidate ray of a pixel. The same FP32 numbers
// enter the same min/max, so the two kernels use bitwise-identical matrix
// entries and <P f, q> = <f, P^T q> holds up to summation order.
//
// Forward: one lane per ray, lanes = consecutive bins of one view (adjacent
// rays walk neighbouring pixels, writes are coalesced). Transpose: one lane
// per pixel, a deterministic gather over views and the pixel's candidate
// bins (no floating-point atomics).
#include "devutil.h"
#include "internal.h"

namespace tnlm {

__device__ __forceinline__ float plane_t(int k, float A, float B) { return fmaf((float)k, A, B); }

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_project(DevGeom g, const float *__restrict__ f,
                                                    const float *__restrict__ y, const float *__restrict__ sw,
                                                    float *__restrict__ out, float *__restrict__ out2,
                                                    double *__restrict__ partials, const int *skip) {
    __shared__ double sh[kBlock];
    if (skip_now(skip)) return;
    const int i = blockIdx.z, v = blockIdx.y;
    const int b = blockIdx.x * kBlock + threadIdx.x;
    const int L = g.L;
    float acc = 0.0f;
    size_t ray = ((size_t)i * g.V + v) * g.B + b;
    if (b < g.B) {
        const float4 A = g.rt0[ray];   // Ax, Bx, Ay, By
        const float4 O = g.rt1[ray];   // ox, oy, ux, uy
        const float tx0 = plane_t(0, A.x, A.y), txL = plane_t(L, A.x, A.y);
        const float ty0 = plane_t(0, A.z, A.w), tyL = plane_t(L, A.z, A.w);
        const float tin = fmaxf(fminf(tx0, txL), fminf(ty0, tyL));
        const float tout = fminf(fmaxf(tx0, txL), fmaxf(ty0, tyL));
        if (tout > tin) {
            const int dc = A.x > 0.0f ? 1 : -1, dr = A.z > 0.0f ? 1 : -1;
            const int hc = dc > 0 ? 1 : 0, hr = dr > 0 ? 1 : 0;   // hi plane = c + hc
            // first pixel: estimate from the entry point, then settle it on the
            // plane values themselves (lo plane <= tin < hi plane)
            const float inv = 1.0f / g.D;
            int c = (int)floorf((fmaf(tin, O.z, O.x) - g.X0) * inv);
            int r = (int)floorf((fmaf(tin, O.w, O.y) - g.X0) * inv);
            c = min(max(c, 0), L - 1);
            r = min(max(r, 0), L - 1);
            for (int it = 0; it < 4; ++it) {
                if (plane_t(c + 1 - hc, A.x, A.y) > tin && (unsigned)(c - dc) < (unsigned)L) c -= dc;
                else if (plane_t(c + hc, A.x, A.y) <= tin && (unsigned)(c + dc) < (unsigned)L) c += dc;
                if (plane_t(r + 1 - hr, A.z, A.w) > tin && (unsigned)(r - dr) < (unsigned)L) r -= dr;
                else if (plane_t(r + hr, A.z, A.w) <= tin && (unsigned)(r + dr) < (unsigned)L) r += dr;
            }
            float txl = plane_t(c + 1 - hc, A.x, A.y), txh = plane_t(c + hc, A.x, A.y);
            float tyl = plane_t(r + 1 - hr, A.z, A.w), tyh = plane_t(r + hr, A.z, A.w);
            const float *__restrict__ fi = f + (size_t)i * L * L;
            // each step leaves at least one axis's current cell: <= 2L steps
            for (int it = 0; it < 2 * L + 2; ++it) {
                const float lo = fmaxf(txl, tyl), hi = fminf(txh, tyh);
                const float l = hi - lo;
                if (l > 0.0f) acc = fmaf(l, fi[r * L + c], acc);
                const bool sx = txh <= tyh, sy = tyh <= txh;
                if (sx) {
                    c += dc;
                    if ((unsigned)c >= (unsigned)L) break;
                    txl = txh;
                    txh = plane_t(c + hc, A.x, A.y);
                }
                if (sy) {
                    r += dr;
                    if ((unsigned)r >= (unsigned)L) break;
                    tyl = tyh;
                    tyh = plane_t(r + hr, A.z, A.w);
                }
            }
        }
    }
    double part = 0.0;
    if (b < g.B) {
        if (MODE == PROJ_PLAIN) {
            out[ray] = acc;
        } else if (MODE == PROJ_RESID) {   // r = sw (y - P u), rw = sw r
            const float s = sw[ray];
            const float res = s * (y[ray] - acc);
            out[ray] = res;
            out2[ray] = s * res;
        } else {                           // q = sw P s, partial ||q||^2
            const float qv = sw[ray] * acc;
            out[ray] = qv;
            part = (double)qv * (double)qv;
        }
    }
    if (MODE == PROJ_SCALED) {
        double tot = block_sum_256(part, sh);
        if (threadIdx.x == 0)
            partials[(size_t)i * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = tot;
    }
}

int proj_blocks_per_phase(const DevGeom &g) { return g.V * ((g.B + kBlock - 1) / kBlock); }

void launch_project(const DevGeom &g, int mode, const float *f, const float *y, const float *sw, float *out,
                    float *out2, double *partials, const int *skip, hipStream_t st) {
    dim3 grid((g.B + kBlock - 1) / kBlock, g.V, g.N);
    if (mode == PROJ_PLAIN)
        k_project<PROJ_PLAIN><<<grid, kBlock, 0, st>>>(g, f, y, sw, out, out2, partials, skip);
    else if (mode == PROJ_RESID)
        k_project<PROJ_RESID><<<grid, kBlock, 0, st>>>(g, f, y, sw, out, out2, partials, skip);
    else
        k_project<PROJ_SCALED><<<grid, kBlock, 0, st>>>(g, f, y, sw, out, out2, partials, skip);
}

// ---------------------------------------------------------------------------
// Transpose: pixel-driven gather. For view v the rays crossing pixel p are the
// bins whose fan angle lies within the pixel's angular extent seen from the
// source; a conservative range (circumscribed circle, small margin) is
// enumerated and each candidate's exact clip is computed with plane_t. Rays
// that miss the pixel yield l <= 0 and add nothing.
// ---------------------------------------------------------------------------
constexpr int kBpTile = 16;

__global__ __launch_bounds__(kBlock) void k_backproject(DevGeom g, const float *__restrict__ q,
                                                        float *__restrict__ fout, double *__restrict__ partials,
                                                        const int *skip) {
    __shared__ double sh[kBlock];
    if (skip_now(skip)) return;
    const int i = blockIdx.z;
    const int c = blockIdx.x * kBpTile + threadIdx.x;
    const int r = blockIdx.y * kBpTile + threadIdx.y;
    const int L = g.L, V = g.V, B = g.B;
    const bool inside = c < L && r < L;
    float acc = 0.0f;
    if (inside) {
        const float px = g.X0 + ((float)c + 0.5f) * g.D, py = g.X0 + ((float)r + 0.5f) * g.D;
        const float rho = 0.70710678f * g.D * 1.001f;
        const float inv_dg = 1.0f / g.dgamma;
        const float4 *__restrict__ rt = g.rt0 + (size_t)i * V * B;
        const float *__restrict__ qi = q + (size_t)i * V * B;
        for (int v = 0; v < V; ++v) {
            const float4 vs = g.vt[i * V + v];   // sx, sy, cos th, sin th
            const float dx = px - vs.x, dy = py - vs.y;
            const float ex = -(dx * vs.z + dy * vs.w), ey = dx * vs.w - dy * vs.z;
            const float gam = atan2f(ey, ex);
            const float dist = sqrtf(dx * dx + dy * dy);
            const float u = gam * inv_dg + g.ucenter;
            const float hw = rho / dist * inv_dg + 0.01f;
            const int b0 = max(0, (int)ceilf(u - hw));
            const int b1 = min(B - 1, (int)floorf(u + hw));
            for (int b = b0; b <= b1; ++b) {
                const float4 A = rt[(size_t)v * B + b];
                const float tx0 = plane_t(c, A.x, A.y), tx1 = plane_t(c + 1, A.x, A.y);
                const float ty0 = plane_t(r, A.z, A.w), ty1 = plane_t(r + 1, A.z, A.w);
                const float lo = fmaxf(fminf(tx0, tx1), fminf(ty0, ty1));
                const float hi = fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1));
                const float l = hi - lo;
                if (l > 0.0f) acc = fmaf(l, qi[(size_t)v * B + b], acc);
            }
        }
        fout[((size_t)i * L + r) * L + c] = acc;
    }
    if (partials != nullptr) {
        double tot = block_sum_256(inside ? (double)acc * (double)acc : 0.0, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0)
            partials[(size_t)i * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = tot;
    }
}

int bp_blocks_per_phase(const DevGeom &g) {
    int t = (g.L + kBpTile - 1) / kBpTile;
    return t * t;
}

void launch_backproject(const DevGeom &g, const float *q, float *f, double *partials, const int *skip,
                        hipStream_t st) {
    int t = (g.L + kBpTile - 1) / kBpTile;
    dim3 grid(t, t, g.N), block(kBpTile, kBpTile);
    k_backproject<<<grid, block, 0, st>>>(g, q, f, partials, skip);
}

}  // namespace tnlm
