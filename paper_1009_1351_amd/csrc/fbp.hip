// Filtered back-projection for the initial image (TNLM algorithm box, step 1):
// textbook equiangular fan-beam FBP over a full turn (Kak & Slaney, ch. 3):
//   R'(k) = y(k) SAD cos(g_k);  Q(n) = dgamma * sum_k R'(k) h(n-k)
//   h(0) = 1/(8 dgamma^2), h(odd m) = -1/(2 pi^2 sin^2(m dgamma)), h(even) = 0
//   f(x) = dbeta * sum_views Q(gamma'(x)) / |x - s|^2, linear interpolation in
//   the bin coordinate, dbeta = 2 pi / (views used).
// The host supplies cw[k] = SAD cos(g_k) and hf[m + B - 1] = dgamma h(m).
#include "devutil.h"
#include "internal.h"

namespace tnlm {

__global__ __launch_bounds__(kBlock) void k_fbp_filter(int B, const float *__restrict__ y, const float *__restrict__ cw,
                                                       const float *__restrict__ hf, float *__restrict__ Q) {
    extern __shared__ float rp[];
    const size_t row = blockIdx.x;
    for (int k = threadIdx.x; k < B; k += kBlock) rp[k] = y[row * B + k] * cw[k];
    __syncthreads();
    for (int n = threadIdx.x; n < B; n += kBlock) {
        const float *h = hf + n + B - 1;   // h[-k] = hf[n - k + B - 1]
        double acc = 0.0;                  // signed terms with cancellation: FP64 sum
        for (int k = 0; k < B; ++k) acc = fma((double)rp[k], (double)h[-k], acc);
        Q[row * B + n] = (float)acc;
    }
}

constexpr int kFbpTile = 16;

__global__ __launch_bounds__(kBlock) void k_fbp_backproject(DevGeom g, const float *__restrict__ Q,
                                                            float *__restrict__ f, int all_phases, float dbeta) {
    const int c = blockIdx.x * kFbpTile + threadIdx.x, r = blockIdx.y * kFbpTile + threadIdx.y;
    const int L = g.L, V = g.V, B = g.B;
    if (c >= L || r >= L) return;
    const float px = g.X0 + ((float)c + 0.5f) * g.D, py = g.X0 + ((float)r + 0.5f) * g.D;
    const float inv_dg = 1.0f / g.dgamma;
    const int i0 = all_phases ? 0 : blockIdx.z, i1 = all_phases ? g.N : blockIdx.z + 1;
    double acc = 0.0;   // thousands of signed terms: FP64 sum (runs once per solve)
    for (int i = i0; i < i1; ++i)
        for (int v = 0; v < V; ++v) {
            const float4 vs = g.vt[i * V + v];
            const float dx = px - vs.x, dy = py - vs.y;
            const float ex = -(dx * vs.z + dy * vs.w), ey = dx * vs.w - dy * vs.z;
            const float u = atan2f(ey, ex) * inv_dg + g.ucenter;
            const float fb = floorf(u);
            const int b0 = (int)fb;
            const float fr = u - fb;
            const float *q = Q + ((size_t)i * V + v) * B;
            float qv = 0.0f;
            if (b0 >= 0 && b0 < B) qv += (1.0f - fr) * q[b0];
            if (b0 + 1 >= 0 && b0 + 1 < B) qv += fr * q[b0 + 1];
            acc += (double)(qv / (dx * dx + dy * dy));
        }
    const float val = (float)((double)dbeta * acc);
    if (all_phases) {
        for (int i = 0; i < g.N; ++i) f[((size_t)i * L + r) * L + c] = val;
    } else {
        f[((size_t)blockIdx.z * L + r) * L + c] = val;
    }
}

void launch_fbp(const DevGeom &g, const float *y, const float *hfilt, const float *cosw, float *Q, float *f,
                int all_phases, float /*sad*/, hipStream_t st) {
    k_fbp_filter<<<g.N * g.V, kBlock, g.B * sizeof(float), st>>>(g.B, y, cosw, hfilt, Q);
    const int t = (g.L + kFbpTile - 1) / kFbpTile;
    const int nviews = all_phases ? g.N * g.V : g.V;
    const float dbeta = (float)(2.0 * 3.14159265358979323846 / nviews);
    dim3 grid(t, t, all_phases ? 1 : g.N), block(kFbpTile, kFbpTile);
    k_fbp_backproject<<<grid, block, 0, st>>>(g, Q, f, all_phases, dbeta);
}

}  // namespace tnlm
