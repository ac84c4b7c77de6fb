// Filtered back-projection for the initial image (TNLM algorithm box, step 1):
// textbook equiangular fan-beam FBP over a full turn (Kak & Slaney, ch. 3):
//   R'(k) = y(k) SAD cos(g_k);  Q(n) = dgamma * sum_k R'(k) h(n-k)
//   h(0) = 1/(8 dgamma^2), h(odd m) = -1/(2 pi^2 sin^2(m dgamma)), h(even) = 0
//   f(x) = dbeta * sum_views Q(gamma'(x)) / |x - s|^2, linear interpolation in
//   the bin coordinate, dbeta = 2 pi / (views used).
// The host supplies, per slice, cw[k] = SAD cos(g_k) and hf[m + B - 1] = dgamma h(m).
#include "devutil.h"
#include "internal.h"

namespace tnlm {

// one block per sinogram row (slice, phase, view)
__global__ __launch_bounds__(kBlock) void k_fbp_filter(Batch bt, Stage st, const float *__restrict__ y,
                                                       const float *__restrict__ cw, const float *__restrict__ hf,
                                                       float *__restrict__ Q) {
    extern __shared__ float rp[];
    for (int gb = blockIdx.x, gend = stage_total(st); gb < gend; gb += gridDim.x) {
        const int s = find_slice(st.pre, bt.ns, gb);
        if (bt.skip && bt.skip[s]) continue;
        const SliceDesc sd = bt.sl[s];
        const int B = sd.B;
        const long long row = sd.sino0 + (long long)(gb - st.pre[s]) * B;
        __syncthreads();
        for (int k = threadIdx.x; k < B; k += kBlock) rp[k] = y[row + k] * cw[sd.cw0 + k];
        __syncthreads();
        for (int n = threadIdx.x; n < B; n += kBlock) {
            const float *h = hf + sd.hf0 + n + B - 1;   // h[-k] = hf[n - k + B - 1]
            double acc = 0.0;                           // signed terms with cancellation: FP64 sum
            for (int k = 0; k < B; ++k) acc = fma((double)rp[k], (double)h[-k], acc);
            Q[row + n] = (float)acc;
        }
    }
}

constexpr int kFbpTile = 16;

int fbp_bp_blocks(const SliceDesc &s, int all_phases) {
    const int t = (s.L + kFbpTile - 1) / kFbpTile;
    return (all_phases ? 1 : s.N) * t * t;
}

__global__ __launch_bounds__(kBlock) void k_fbp_backproject(Batch bt, Stage st, const float *__restrict__ Q,
                                                            float *__restrict__ f, int all_phases) {
    const int tx = threadIdx.x % kFbpTile, ty = threadIdx.x / kFbpTile;
    for (int gb = blockIdx.x, gend = stage_total(st); gb < gend; gb += gridDim.x) {
        const int s = find_slice(st.pre, bt.ns, gb);
        if (bt.skip && bt.skip[s]) continue;
        const SliceDesc sd = bt.sl[s];
        const int L = sd.L, V = sd.V, B = sd.B;
        const int nt = (L + kFbpTile - 1) / kFbpTile;
        int lb = gb - st.pre[s];
        const int tcx = lb % nt;
        lb /= nt;
        const int tcy = lb % nt, img = lb / nt;
        const int c = tcx * kFbpTile + tx, r = tcy * kFbpTile + ty;
        if (c >= L || r >= L) continue;
        const float px = sd.X0 + ((float)c + 0.5f) * sd.D, py = sd.X0 + ((float)r + 0.5f) * sd.D;
        const float inv_dg = 1.0f / sd.dgamma;
        const int i0 = all_phases ? 0 : img, i1 = all_phases ? sd.N : img + 1;
        const double dbeta = 2.0 * 3.14159265358979323846 / (double)(all_phases ? sd.N * V : V);
        double acc = 0.0;   // thousands of signed terms: FP64 sum (runs once per solve)
        for (int i = i0; i < i1; ++i)
            for (int v = 0; v < V; ++v) {
                const float4 vs = bt.vt[sd.view0 + (long long)i * V + v];
                const float dx = px - vs.x, dy = py - vs.y;
                const float ex = -(dx * vs.z + dy * vs.w), ey = dx * vs.w - dy * vs.z;
                const float u = atan2f(ey, ex) * inv_dg + sd.ucenter;
                const float fb = floorf(u);
                const int b0 = (int)fb;
                const float fr = u - fb;
                const float *q = Q + sd.sino0 + ((long long)i * V + v) * B;
                float qv = 0.0f;
                if (b0 >= 0 && b0 < B) qv += (1.0f - fr) * q[b0];
                if (b0 + 1 >= 0 && b0 + 1 < B) qv += fr * q[b0 + 1];
                acc += (double)(qv / (dx * dx + dy * dy));
            }
        const float val = (float)(dbeta * acc);
        if (all_phases) {
            for (int i = 0; i < sd.N; ++i) f[sd.img0 + ((long long)i * L + r) * L + c] = val;
        } else {
            f[sd.img0 + ((long long)img * L + r) * L + c] = val;
        }
    }
}

void launch_fbp(const Batch &b, const Stage &filt, const Stage &bp, const float *y, const float *hfilt,
                const float *cosw, float *Q, float *f, int all_phases, hipStream_t strm) {
    if (filt.total == 0) return;
    k_fbp_filter<<<filt.grid, kBlock, 4096 * sizeof(float), strm>>>(b, filt, y, cosw, hfilt, Q);
    k_fbp_backproject<<<bp.grid, kBlock, 0, strm>>>(b, bp, Q, f, all_phases);
}

}  // namespace tnlm
