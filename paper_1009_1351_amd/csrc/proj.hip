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
// bins (no floating-point atomics). Both are persistent over the batch's
// ragged slice table.
#include "devutil.h"
#include "internal.h"

namespace tnlm {

__device__ __forceinline__ float plane_t(int k, float A, float B) { return fmaf((float)k, A, B); }

constexpr int kRaysPerBlock = kBlock;

int proj_blocks(const SliceDesc &s) { return s.N * s.V * ((s.B + kRaysPerBlock - 1) / kRaysPerBlock); }

// One ray: Siddon walk of image fi (L x L) along plane table A and ray point/direction O.
__device__ __forceinline__ float walk_ray(const float4 A, const float4 O, const float *__restrict__ fi, int L,
                                          float X0, float invD) {
    const float tx0 = plane_t(0, A.x, A.y), txL = plane_t(L, A.x, A.y);
    const float ty0 = plane_t(0, A.z, A.w), tyL = plane_t(L, A.z, A.w);
    const float tin = fmaxf(fminf(tx0, txL), fminf(ty0, tyL));
    const float tout = fminf(fmaxf(tx0, txL), fmaxf(ty0, tyL));
    float acc = 0.0f;
    if (!(tout > tin)) return acc;
    const int dc = A.x > 0.0f ? 1 : -1, dr = A.z > 0.0f ? 1 : -1;
    const int hc = dc > 0 ? 1 : 0, hr = dr > 0 ? 1 : 0;   // hi plane of cell c = c + hc
    // first cell: estimate from the entry point, then settle it on the plane
    // values themselves (lo plane <= tin < hi plane)
    int c = (int)floorf((fmaf(tin, O.z, O.x) - X0) * invD);
    int r = (int)floorf((fmaf(tin, O.w, O.y) - X0) * invD);
    c = min(max(c, 0), L - 1);
    r = min(max(r, 0), L - 1);
    for (int it = 0; it < 4; ++it) {
        if (plane_t(c + 1 - hc, A.x, A.y) > tin && (unsigned)(c - dc) < (unsigned)L) c -= dc;
        else if (plane_t(c + hc, A.x, A.y) <= tin && (unsigned)(c + dc) < (unsigned)L) c += dc;
        if (plane_t(r + 1 - hr, A.z, A.w) > tin && (unsigned)(r - dr) < (unsigned)L) r -= dr;
        else if (plane_t(r + hr, A.z, A.w) <= tin && (unsigned)(r + dr) < (unsigned)L) r += dr;
    }
    // Walk: tcur is the lo plane of the current cell (max of its x/y lo
    // planes); the next crossing is min(txh, tyh). Each segment equals the
    // clip of the cell computed by the transpose kernel, bit for bit.
    float fkx = (float)(c + hc), fky = (float)(r + hr);
    float txh = plane_t(c + hc, A.x, A.y), tyh = plane_t(r + hr, A.z, A.w);
    float tcur = fmaxf(plane_t(c + 1 - hc, A.x, A.y), plane_t(r + 1 - hr, A.z, A.w));
    const float dcf = (float)dc, drf = (float)dr;
    const int sx_ofs = dc, sy_ofs = dr * L;
    int idx = r * L + c;
    // every step moves past at least one grid line: at most 2L + 1 cells
    for (int it = 0; it < 2 * L + 2; ++it) {
        const float tn = fminf(txh, tyh);
        acc = fmaf(tn - tcur, fi[idx], acc);
        if (!(tn < tout)) break;   // the cell just added was the last one
        tcur = tn;
        const bool sx = txh <= tyh, sy = tyh <= txh;
        fkx += sx ? dcf : 0.0f;
        fky += sy ? drf : 0.0f;
        idx += (sx ? sx_ofs : 0) + (sy ? sy_ofs : 0);
        if ((unsigned)idx >= (unsigned)(L * L)) break;   // memory guard; never taken
        txh = sx ? fmaf(fkx, A.x, A.y) : txh;
        tyh = sy ? fmaf(fky, A.z, A.w) : tyh;
    }
    return acc;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_project(Batch bt, Stage st, const float *__restrict__ f,
                                                    const float *__restrict__ y, const float *__restrict__ sw,
                                                    float *__restrict__ out, float *__restrict__ out2,
                                                    double *__restrict__ partials) {
    __shared__ double sh[kBlock];
    int first, stride, count;
    xcd_range(st.total, first, stride, count);
    for (int gb = first; gb < count; gb += stride) {
        const int s = find_slice(st.pre, bt.ns, gb);
        if (bt.skip && bt.skip[s]) continue;
        const SliceDesc sd = bt.sl[s];
        const int nbx = (sd.B + kRaysPerBlock - 1) / kRaysPerBlock;
        int lb = gb - st.pre[s];
        const int bx = lb % nbx;
        lb /= nbx;
        const int v = lb % sd.V, i = lb / sd.V;
        const int b = bx * kRaysPerBlock + threadIdx.x;
        const long long ray = ((long long)i * sd.V + v) * sd.B + b;   // within the slice
        float acc = 0.0f;
        if (b < sd.B)
            acc = walk_ray(bt.rt0[sd.ray0 + ray], bt.rt1[sd.ray0 + ray], f + sd.img0 + (long long)i * sd.L * sd.L,
                           sd.L, sd.X0, 1.0f / sd.D);
        double part = 0.0;
        if (b < sd.B) {
            const long long e = sd.sino0 + ray;
            if (MODE == PROJ_PLAIN) {
                out[e] = acc;
            } else if (MODE == PROJ_RESID) {   // r = sw (y - P u), rw = sw r
                const float w = sw[e];
                const float res = w * (y[e] - acc);
                out[e] = res;
                out2[e] = w * res;
            } else {                           // q = sw P s, partial ||q||^2
                const float qv = sw[e] * acc;
                out[e] = qv;
                part = (double)qv * (double)qv;
            }
        }
        if (MODE == PROJ_SCALED) {
            const double tot = block_sum_256(part, sh);
            if (threadIdx.x == 0) partials[sd.qp0 + (long long)i * sd.npp + v * nbx + bx] = tot;
        }
    }
}

void launch_project(const Batch &b, const Stage &st, int mode, const float *f, const float *y, const float *sw,
                    float *out, float *out2, double *partials, hipStream_t strm) {
    if (st.total == 0) return;
    if (mode == PROJ_PLAIN)
        k_project<PROJ_PLAIN><<<st.grid, kBlock, 0, strm>>>(b, st, f, y, sw, out, out2, partials);
    else if (mode == PROJ_RESID)
        k_project<PROJ_RESID><<<st.grid, kBlock, 0, strm>>>(b, st, f, y, sw, out, out2, partials);
    else
        k_project<PROJ_SCALED><<<st.grid, kBlock, 0, strm>>>(b, st, f, y, sw, out, out2, partials);
}

// ---------------------------------------------------------------------------
// Transpose: pixel-driven gather. For view v the rays crossing pixel p are the
// bins whose fan angle lies within the pixel's angular extent seen from the
// source; a conservative range is enumerated and each candidate's exact clip
// is computed with plane_t. Rays that miss the pixel add l = 0.
// ---------------------------------------------------------------------------
constexpr int kBpTile = 16;

// atan(t) for |t| <= 0.62 (|angle| <= 0.555 rad, beyond the fan half-angle of
// the scanner): t * p(t^2), p of degree 4 fitted by weighted least squares on
// Chebyshev nodes; max error 1.9e-7 rad. Only used to enumerate candidate bins.
__device__ __forceinline__ float fan_atan(float t) {
    const float s = t * t;
    float p = fmaf(s, 0.05211811f, -0.12408195f);
    p = fmaf(s, p, 0.19714545f);
    p = fmaf(s, p, -0.33315012f);
    p = fmaf(s, p, 0.99999666f);
    return t * p;
}

int bp_blocks(const SliceDesc &s) {
    const int t = (s.L + kBpTile - 1) / kBpTile;
    return s.N * t * t;
}

__global__ __launch_bounds__(kBlock) void k_backproject(Batch bt, Stage st, const float *__restrict__ q,
                                                        float *__restrict__ fout, double *__restrict__ partials) {
    __shared__ double sh[kBlock];
    int first, stride, count;
    xcd_range(st.total, first, stride, count);
    const int tx = threadIdx.x % kBpTile, ty = threadIdx.x / kBpTile;
    for (int gb = first; gb < count; gb += stride) {
        const int s = find_slice(st.pre, bt.ns, gb);
        if (bt.skip && bt.skip[s]) continue;
        const SliceDesc sd = bt.sl[s];
        const int L = sd.L, V = sd.V, B = sd.B;
        const int nt = (L + kBpTile - 1) / kBpTile;
        int lb = gb - st.pre[s];
        const int tcx = lb % nt;
        lb /= nt;
        const int tcy = lb % nt, i = lb / nt;
        const int c = tcx * kBpTile + tx, r = tcy * kBpTile + ty;
        const bool inside = c < L && r < L;
        float acc = 0.0f;
        if (inside) {
            const float px = sd.X0 + ((float)c + 0.5f) * sd.D, py = sd.X0 + ((float)r + 0.5f) * sd.D;
            const float half = 0.5f * sd.D;
            const float inv_dg = 1.0f / sd.dgamma;
            const float4 *__restrict__ rt = bt.rt0 + sd.ray0 + (long long)i * V * B;
            const float4 *__restrict__ vt = bt.vt + sd.view0 + (long long)i * V;
            const float *__restrict__ qi = q + sd.sino0 + (long long)i * V * B;
            for (int v = 0; v < V; ++v) {
                const float4 vs = vt[v];   // sx, sy, cos th, sin th
                const float dx = px - vs.x, dy = py - vs.y;
                // (ex, ey): pixel centre in the frame of the central ray
                const float ex = -(dx * vs.z + dy * vs.w), ey = dx * vs.w - dy * vs.z;
                const float inv_dist = rsqrtf(dx * dx + dy * dy);
                const float tq = ey * __builtin_amdgcn_rcpf(ex);
                const float gam = (ex > 0.0f && fabsf(tq) <= 0.62f) ? fan_atan(tq) : atan2f(ey, ex);
                // angular half-width of the pixel seen from the source: half-extent
                // w of the square across the ray over the distance, a second-order
                // bound for the nearer corners, and a small margin in bins
                const float wq = half * (fabsf(dx) + fabsf(dy)) * inv_dist * inv_dist;
                const float u = gam * inv_dg + sd.ucenter;
                const float hw = wq * (1.0f + 2.0f * wq) * 1.01f * inv_dg + 0.01f;
                const int b0 = max(0, (int)ceilf(u - hw));
                const int b1 = min(B - 1, (int)floorf(u + hw));
                for (int b = b0; b <= b1; ++b) {
                    const float4 A = rt[(long long)v * B + b];
                    const float tx0 = plane_t(c, A.x, A.y), tx1 = plane_t(c + 1, A.x, A.y);
                    const float ty0 = plane_t(r, A.z, A.w), ty1 = plane_t(r + 1, A.z, A.w);
                    const float lo = fmaxf(fminf(tx0, tx1), fminf(ty0, ty1));
                    const float hi = fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1));
                    acc = fmaf(fmaxf(hi - lo, 0.0f), qi[(long long)v * B + b], acc);
                }
            }
            fout[sd.img0 + ((long long)i * L + r) * L + c] = acc;
        }
        if (partials != nullptr) {
            const double tot = block_sum_256(inside ? (double)acc * (double)acc : 0.0, sh);
            if (threadIdx.x == 0) partials[sd.gp0 + (long long)i * sd.nbp + tcy * nt + tcx] = tot;
        }
    }
}

void launch_backproject(const Batch &b, const Stage &st, const float *q, float *f, double *partials,
                        hipStream_t strm) {
    if (st.total == 0) return;
    k_backproject<<<st.grid, kBlock, 0, strm>>>(b, st, q, f, partials);
}

}  // namespace tnlm
