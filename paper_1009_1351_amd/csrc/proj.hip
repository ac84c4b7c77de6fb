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
// Forward: one lane per ray, lanes = consecutive bins of one view, walking
// the image row by row in step (adjacent rays read neighbouring pixels of one
// row, writes are coalesced). Transpose: one lane
// per pixel, a deterministic gather over views and the pixel's candidate
// bins (no floating-point atomics). Both are persistent over the batch's
// ragged slice table.
#include "devutil.h"
#include "internal.h"

namespace tnlm {

__device__ __forceinline__ float plane_t(int k, float A, float B) { return fmaf((float)k, A, B); }

constexpr int kRaysPerBlock = kBlock;

int proj_blocks(const SliceDesc &s) { return s.N * s.V * ((s.B + kRaysPerBlock - 1) / kRaysPerBlock); }

// Image reads of the walk go through a buffer resource spanning one phase
// image: an offset outside it reads 0 without a memory access (the walk
// prefetches the cell after the current one, which lies outside the image
// once the ray leaves it).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const float *fi, int L) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(fi), (short)0, L * L * 4, 0x00020000);
}

__device__ __forceinline__ float image_at(__amdgpu_buffer_rsrc_t img, int byte_off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(img, byte_off, 0, 0));
}

__device__ __forceinline__ float cell_clip(float xl, float xh, float yl, float yh) {
    return fmaxf(fminf(xh, yh) - fmaxf(xl, yl), 0.0f);
}

// Offset that the image's buffer resource turns into a read of 0 without a
// memory access (beyond the L x L image for every L the engine accepts).
constexpr int kNoCell = 0x40000000;

// Row-synchronous walk of one wave's rays over one phase image (L x L). The
// plane tables A (x planes in .x/.y, y planes in .z/.w) and ray points O come
// in the wave's frame, in which every ray of the wave crosses about one
// column per row or fewer. Pass p visits image row p counted along the rays'
// row direction for all lanes at once, so the lanes of a wave read
// neighbouring cells of one row (two per lane: the current column and the
// next) rather than drifting apart by their different numbers of column
// crossings. The length of each cell is the clip of the transpose kernel and
// cells are added in the order the ray meets them (a ray that reaches the next
// column exactly at the row's upper plane enters it with length 0 first), so
// the sum is bitwise that of a walk crossing one grid line at a time. The wave
// runs from the first entry row to the last exit row of its rays; a lane that
// leaves through a side stops adding there, and a ray crossing two columns in
// one row takes the rare inner loop.
// Must be called by all lanes of the wave; lanes with valid = false add nothing.
__device__ __forceinline__ float walk_rows(const float4 A, const float4 O, bool valid,
                                           __amdgpu_buffer_rsrc_t img, int L, float X0, float invD) {
    int pin = L, pout = -1, c = 0, dc = 1, dr = 1, hc = 1, hr = 1;
    float tin = 0.0f;
    bool hit = false;
    if (valid) {
        const float tx0 = plane_t(0, A.x, A.y), txL = plane_t(L, A.x, A.y);
        const float ty0 = plane_t(0, A.z, A.w), tyL = plane_t(L, A.z, A.w);
        tin = fmaxf(fminf(tx0, txL), fminf(ty0, tyL));
        const float tout = fminf(fmaxf(tx0, txL), fmaxf(ty0, tyL));
        if (tout > tin) {
            hit = true;
            dc = A.x > 0.0f ? 1 : -1;
            dr = A.z > 0.0f ? 1 : -1;
            hc = dc > 0 ? 1 : 0;   // hi plane of cell c = c + hc
            hr = dr > 0 ? 1 : 0;
            // entry cell: estimate from the entry point, then settle it on the
            // plane values themselves (lo plane <= tin < hi plane)
            c = (int)floorf((fmaf(tin, O.z, O.x) - X0) * invD);
            int r = (int)floorf((fmaf(tin, O.w, O.y) - X0) * invD);
            c = min(max(c, 0), L - 1);
            r = min(max(r, 0), L - 1);
            for (int it = 0; it < 4; ++it) {
                if (plane_t(c + 1 - hc, A.x, A.y) > tin && (unsigned)(c - dc) < (unsigned)L) c -= dc;
                else if (plane_t(c + hc, A.x, A.y) <= tin && (unsigned)(c + dc) < (unsigned)L) c += dc;
                if (plane_t(r + 1 - hr, A.z, A.w) > tin && (unsigned)(r - dr) < (unsigned)L) r -= dr;
                else if (plane_t(r + hr, A.z, A.w) <= tin && (unsigned)(r + dr) < (unsigned)L) r += dr;
            }
            pin = dr > 0 ? r : L - 1 - r;   // pass of the entry row
            // pass of the exit row, from the exit point, with two rows of
            // margin for its rounding (rows past the exit add nothing)
            int re = (int)floorf((fmaf(tout, O.w, O.y) - X0) * invD);
            re = min(max(re, 0), L - 1);
            pout = min((dr > 0 ? re : L - 1 - re) + 2, L - 1);
        }
    }
    int p0 = pin, p1 = pout;   // first and last pass of the wave
    for (int m = 32; m > 0; m >>= 1) {
        p0 = min(p0, __shfl_xor(p0, m, 64));
        p1 = max(p1, __shfl_xor(p1, m, 64));
    }
    p0 = wave_uniform(p0);
    p1 = wave_uniform(p1);
    const int r0 = dr > 0 ? p0 : L - 1 - p0;
    const float dcf = (float)dc, drf = (float)dr;
    const int ox = 4 * dc, oy = 4 * dr * L;
    float fkx = (float)(c + hc), fky = (float)(r0 + hr);
    float txh = plane_t(c + hc, A.x, A.y);
    float tyl = plane_t(r0 + 1 - hr, A.z, A.w);
    int rowoff = 4 * r0 * L;
    bool dead = !hit;
    bool live = hit && p0 >= pin;
    int o1 = live ? rowoff + 4 * c : kNoCell;
    float v1 = image_at(img, o1), v2 = image_at(img, o1 + ox);
    float acc = 0.0f;
    for (int p = p0; p <= p1; ++p) {
        // At the start of a row a live lane's column c holds its ray and the
        // column's upper x plane lies beyond the row's lower y plane
        // (txh > tyl), so the clip of (r, c) is non-negative and that of
        // (r, c + dc) has max(txh, tyl) = txh: both are the transpose
        // kernel's clips without its clamp. The lower x plane of column c
        // is at most tyl in every row but the entry row, where it is tin or
        // at most tin = tyl, so max(x_lo, tyl) = max(tin, tyl) throughout.
        // Lanes that are not live read 0.
        const float tyh = fmaf(fky, A.z, A.w);
        const float txn = fmaf(fkx + dcf, A.x, A.y);
        const float l1 = fminf(txh, tyh) - fmaxf(tin, tyl);
        const float l2 = fminf(txn, tyh) - txh;
        const bool cross = live && txh <= tyh;   // reaches the next column in this row
        const bool in2 = (unsigned)(c + dc) < (unsigned)L;
        const bool take2 = cross && in2;
        acc = fmaf(l1, v1, acc);
        acc = fmaf(take2 ? l2 : 0.0f, v2, acc);
        dead = dead || (cross && !in2);   // left the image through a side
        c = take2 ? c + dc : c;
        fkx = take2 ? fkx + dcf : fkx;
        txh = take2 ? txn : txh;
        while (take2 && txh <= tyh) {   // a further column in the same row
            if ((unsigned)(c + dc) >= (unsigned)L) {
                dead = true;
                break;
            }
            const float tx3 = fmaf(fkx + dcf, A.x, A.y);
            acc = fmaf(cell_clip(txh, tx3, tyl, tyh), image_at(img, rowoff + 4 * (c + dc)), acc);
            c += dc;
            fkx += dcf;
            txh = tx3;
        }
        tyl = tyh;
        fky += drf;
        rowoff += oy;
        live = !dead && p + 1 >= pin;
        o1 = live ? rowoff + 4 * c : kNoCell;
        v1 = image_at(img, o1);   // next row's cells, in flight during the next pass's plane arithmetic
        v2 = image_at(img, o1 + ox);
    }
    return acc;
}

// Image stacks are row-major, (r, c) at r L + c. A projector wave walks rows
// in step, which suits rays that run mostly along y: its lanes then sit in
// one row at neighbouring columns (few cache lines per load). A wave whose
// rays run mostly along x walks a transposed copy, (r, c) at c L + r, with
// the roles of the axes exchanged; the cells and their lengths are the same
// (at a grid corner the zero-length cell passed through is the other one), so
// the sum is bitwise the same for a finite image.
constexpr int kTr = 32;

int tr_blocks(const SliceDesc &s) {
    const int t = (s.L + kTr - 1) / kTr;
    return s.N * t * t;
}

__global__ __launch_bounds__(kBlock) void k_transpose(Batch bt, Stage st, const float *__restrict__ f,
                                                      float *__restrict__ fT) {
    __shared__ float tile[kTr][kTr + 1];
    int first, stride, count;
    xcd_range(st, first, stride, count);
    const int tx = threadIdx.x % kTr, ty = threadIdx.x / kTr;   // 32 x 8
    for (int gb = first; gb < count; gb += stride) {
        const int s = find_slice(st.pre, bt.ns, gb);
        if (bt.skip && bt.skip[s]) continue;
        const SliceDesc sd = load_const(bt.sl, s);
        const int L = sd.L, t = (L + kTr - 1) / kTr;
        int lb = gb - load_const(st.pre, s);
        const int bx = lb % t;
        lb /= t;
        const int by = lb % t, i = lb / t;
        const float *__restrict__ src = f + sd.img0 + (long long)i * L * L;
        float *__restrict__ dst = fT + sd.img0 + (long long)i * L * L;
        for (int k = 0; k < kTr; k += kBlock / kTr) {
            const int r = by * kTr + ty + k, c = bx * kTr + tx;
            if (r < L && c < L) tile[ty + k][tx] = src[r * L + c];
        }
        __syncthreads();
        for (int k = 0; k < kTr; k += kBlock / kTr) {
            const int c = bx * kTr + ty + k, r = by * kTr + tx;
            if (r < L && c < L) dst[c * L + r] = tile[tx][ty + k];
        }
        __syncthreads();
    }
}

void launch_transpose(const Batch &b, const Stage &st, const float *f, float *fT, hipStream_t strm) {
    if (st.total == 0) return;
    k_transpose<<<st.grid, kBlock, 0, strm>>>(b, st, f, fT);
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_project(Batch bt, Stage st, const float *__restrict__ f,
                                                    const float *__restrict__ fT, const float *__restrict__ y,
                                                    const float *__restrict__ sw, float *__restrict__ out,
                                                    float *__restrict__ out2, double *__restrict__ partials) {
    __shared__ double sh[kBlock];
    __shared__ int sh_item;
    WorkIter it = work_begin(st);
    int gb;
    while (work_next(st, it, gb, &sh_item)) {
        const int s = find_slice(st.pre, bt.ns, gb);
        if (bt.skip && bt.skip[s]) continue;
        const SliceDesc sd = load_const(bt.sl, s);
        const int nbx = (sd.B + kRaysPerBlock - 1) / kRaysPerBlock;
        int lb = gb - st.pre[s];
        const int bx = lb % nbx;
        lb /= nbx;
        const int v = lb % sd.V, i = lb / sd.V;
        const int b = bx * kRaysPerBlock + threadIdx.x;
        const long long ray = ((long long)i * sd.V + v) * sd.B + b;   // within the slice
        const int L = sd.L;
        const bool valid = b < sd.B;
        float4 A = make_float4(1.0f, 0.0f, 1.0f, 0.0f), O = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
        if (valid) {
            A = bt.rt0[sd.ray0 + ray];
            O = bt.rt1[sd.ray0 + ray];
        }
        // the wave walks the transposed image, axes exchanged, when most of
        // its rays cross columns faster than rows
        const bool xmaj = valid && fabsf(A.x) < fabsf(A.z);
        const bool tr = wave_uniform(2 * __popcll(__ballot(xmaj)) > __popcll(__ballot(valid)));
        if (tr) {
            A = make_float4(A.z, A.w, A.x, A.y);
            O = make_float4(O.y, O.x, O.w, O.z);
        }
        const __amdgpu_buffer_rsrc_t img = image_rsrc((tr ? fT : f) + sd.img0 + (long long)i * L * L, L);
        const float acc = walk_rows(A, O, valid, img, L, sd.X0, 1.0f / sd.D);
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
    work_end(st);
}

void launch_project(const Batch &b, const Stage &st, int mode, const float *f, const float *fT, const float *y,
                    const float *sw, float *out, float *out2, double *partials, hipStream_t strm) {
    if (st.total == 0) return;
    if (mode == PROJ_PLAIN)
        k_project<PROJ_PLAIN><<<st.grid, kBlock, 0, strm>>>(b, st, f, fT, y, sw, out, out2, partials);
    else if (mode == PROJ_RESID)
        k_project<PROJ_RESID><<<st.grid, kBlock, 0, strm>>>(b, st, f, fT, y, sw, out, out2, partials);
    else
        k_project<PROJ_SCALED><<<st.grid, kBlock, 0, strm>>>(b, st, f, fT, y, sw, out, out2, partials);
}

// ---------------------------------------------------------------------------
// Transpose: pixel-driven gather. For view v the rays crossing pixel p are the
// bins whose fan angle lies within the pixel's angular extent seen from the
// source; a conservative range is enumerated and each candidate's exact clip
// is computed with plane_t. Rays that miss the pixel add l = 0.
// ---------------------------------------------------------------------------
// Each lane gathers a 2 x 2 block of pixels; a block of 256 lanes covers a
// 32 x 32 tile. The candidate bins of a view are those of the 2 x 2 square
// (a superset of each pixel's own), found once per lane and view; the three
// x-planes and three y-planes of the square serve its four pixels. A
// candidate ray that misses a pixel adds exactly zero, so every pixel
// receives the same contributions in the same order as a gather over its
// own candidate range.
constexpr int kBpTile = 32;
constexpr int kBpLanes = kBpTile / 2;   // lanes per tile side

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

// Candidate loop of one lane and view with the direction signs of all
// candidate rays fixed (XP: T_x grows with the plane index; YP likewise):
// planes c, c+1, c+2 (and r, r+1, r+2) are evaluated once and take the lo or
// hi role of each pixel by the signs.
template <bool XP, bool YP>
__device__ __forceinline__ void bp_block_ray(const float4 A, const float qb, float fc0, float fr0, float &a00,
                                             float &a01, float &a10, float &a11) {
    const float fc1 = fc0 + 1.0f, fc2 = fc0 + 2.0f, fr1 = fr0 + 1.0f, fr2 = fr0 + 2.0f;
    const float X0 = fmaf(fc0, A.x, A.y), X1 = fmaf(fc1, A.x, A.y), X2 = fmaf(fc2, A.x, A.y);
    const float Y0 = fmaf(fr0, A.z, A.w), Y1 = fmaf(fr1, A.z, A.w), Y2 = fmaf(fr2, A.z, A.w);
    const float xl0 = XP ? X0 : X1, xh0 = XP ? X1 : X0;   // column c
    const float xl1 = XP ? X1 : X2, xh1 = XP ? X2 : X1;   // column c + 1
    const float yl0 = YP ? Y0 : Y1, yh0 = YP ? Y1 : Y0;   // row r
    const float yl1 = YP ? Y1 : Y2, yh1 = YP ? Y2 : Y1;   // row r + 1
    a00 = fmaf(fmaxf(fminf(xh0, yh0) - fmaxf(xl0, yl0), 0.0f), qb, a00);
    a01 = fmaf(fmaxf(fminf(xh1, yh0) - fmaxf(xl1, yl0), 0.0f), qb, a01);
    a10 = fmaf(fmaxf(fminf(xh0, yh1) - fmaxf(xl0, yl1), 0.0f), qb, a10);
    a11 = fmaf(fmaxf(fminf(xh1, yh1) - fmaxf(xl1, yl1), 0.0f), qb, a11);
}

// Two candidates per pass, both requested before either is used; an odd last
// candidate takes a pass of its own, so the additions happen in the same order
// as one candidate per pass. The view's plane records and sinogram values are
// read through buffer resources (wave-uniform bases) at per-lane 32-bit
// offsets: one offset step per pass instead of 64-bit address arithmetic.
__device__ __forceinline__ float4 rsrc_f4(__amdgpu_buffer_rsrc_t r, int off) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
}

template <bool XP, bool YP>
__device__ __forceinline__ void bp_block_oriented(__amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rq, int b0,
                                                  int b1, float fc0, float fr0, float &a00, float &a01, float &a10,
                                                  float &a11) {
    int off = 16 * b0;          // byte offset of the candidate's plane record
    const int last = 16 * b1;   // that of the last candidate
    for (; off < last; off += 32) {   // at least two candidates left
        const float4 A = rsrc_f4(ra, off), An = rsrc_f4(ra, off + 16);
        const float qb = image_at(rq, off >> 2), qn = image_at(rq, (off >> 2) + 4);
        bp_block_ray<XP, YP>(A, qb, fc0, fr0, a00, a01, a10, a11);
        bp_block_ray<XP, YP>(An, qn, fc0, fr0, a00, a01, a10, a11);
    }
    if (off == last) bp_block_ray<XP, YP>(rsrc_f4(ra, off), image_at(rq, off >> 2), fc0, fr0, a00, a01, a10, a11);
}

int bp_blocks(const SliceDesc &s) {
    const int t = (s.L + kBpTile - 1) / kBpTile;
    return s.N * t * t;
}

__global__ __launch_bounds__(kBlock) void k_backproject(Batch bt, Stage st, const float *__restrict__ q,
                                                        float *__restrict__ fout, double *__restrict__ partials) {
    __shared__ double sh[kBlock];
    __shared__ int sh_item;
    WorkIter it = work_begin(st);
    int gb;
    const int tx = threadIdx.x % kBpLanes, ty = threadIdx.x / kBpLanes;
    while (work_next(st, it, gb, &sh_item)) {
        const int s = find_slice(st.pre, bt.ns, gb);
        if (bt.skip && bt.skip[s]) continue;
        const SliceDesc sd = load_const(bt.sl, s);
        const int L = sd.L, V = sd.V, B = sd.B;
        const int nt = (L + kBpTile - 1) / kBpTile;
        int lb = gb - st.pre[s];
        const int tcx = lb % nt;
        lb /= nt;
        const int tcy = lb % nt, i = lb / nt;
        const int c = tcx * kBpTile + 2 * tx, r = tcy * kBpTile + 2 * ty;   // lower-left pixel of the 2 x 2 block
        const bool any = c < L && r < L;
        float a00 = 0.0f, a01 = 0.0f, a10 = 0.0f, a11 = 0.0f;   // a<row><col>
        if (any) {
            // centre of the 2 x 2 square (a grid corner) and its half-side D
            const float px = sd.X0 + (float)(c + 1) * sd.D, py = sd.X0 + (float)(r + 1) * sd.D;
            const float inv_dg = 1.0f / sd.dgamma;
            const float wscale = sd.D * 1.01f * inv_dg;
            const float4 *__restrict__ rt = bt.rt0 + sd.ray0 + (long long)i * V * B;
            const float *__restrict__ qi = q + sd.sino0 + (long long)i * V * B;
            const long long v0 = sd.view0 + (long long)i * V;
            const float fc0 = (float)c, fc1 = (float)(c + 1), fc2 = (float)(c + 2);
            const float fr0 = (float)r, fr1 = (float)(r + 1), fr2 = (float)(r + 2);
            for (int v = 0; v < V; ++v) {
                const float4 vs = load_const(bt.vt, v0 + v);   // sx, sy, cos th, sin th
                const int4 vb = load_const(bt.vo, v0 + v);     // sign changes of Ax, Ay over the bins
                const float dx = px - vs.x, dy = py - vs.y;
                // (ex, ey): square centre in the frame of the central ray
                const float ex = -(dx * vs.z + dy * vs.w), ey = dx * vs.w - dy * vs.z;
                const float inv_dist = __builtin_amdgcn_rsqf(dx * dx + dy * dy);
                const float tq = ey * __builtin_amdgcn_rcpf(ex);
                const float gam = (ex > 0.0f && fabsf(tq) <= 0.62f) ? fan_atan(tq) : atan2f(ey, ex);
                // angular half-width of the square seen from the source: its
                // half-extent across the ray over the distance, a second-order
                // bound for the nearer corners, and a small margin in bins
                const float wq = (fabsf(dx) + fabsf(dy)) * inv_dist * inv_dist;   // over the half-side
                const float u = fmaf(gam, inv_dg, sd.ucenter);
                const float hw = fmaf(wq * wscale, fmaf(wq, 2.0f * sd.D, 1.0f), 0.01f);
                const int b0 = max(0, (int)ceilf(u - hw));
                const int b1 = min(B - 1, (int)floorf(u + hw));
                const float4 *__restrict__ Av = rt + (long long)v * B;
                const float *__restrict__ qv = qi + (long long)v * B;
                if (!((b0 < vb.x && b1 >= vb.x) || (b0 < vb.y && b1 >= vb.y))) {
                    // every candidate ray has the same direction signs: the lo and
                    // hi plane of each pixel along each axis are known, and the clip
                    // max(min(..), min(..)) / min(max(..), max(..)) reduces to one
                    // comparison per side (the same values as the general form)
                    const bool xpos = ((vb.z & 1) != 0) == (b0 < vb.x);
                    const bool ypos = ((vb.z & 2) != 0) == (b0 < vb.y);
                    const __amdgpu_buffer_rsrc_t ra =
                        __builtin_amdgcn_make_buffer_rsrc(const_cast<float4 *>(Av), (short)0, B * 16, 0x00020000);
                    const __amdgpu_buffer_rsrc_t rq =
                        __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(qv), (short)0, B * 4, 0x00020000);
                    if (xpos) {
                        if (ypos) bp_block_oriented<true, true>(ra, rq, b0, b1, fc0, fr0, a00, a01, a10, a11);
                        else bp_block_oriented<true, false>(ra, rq, b0, b1, fc0, fr0, a00, a01, a10, a11);
                    } else {
                        if (ypos) bp_block_oriented<false, true>(ra, rq, b0, b1, fc0, fr0, a00, a01, a10, a11);
                        else bp_block_oriented<false, false>(ra, rq, b0, b1, fc0, fr0, a00, a01, a10, a11);
                    }
                } else {
                    for (int b = b0; b <= b1; ++b) {
                        const float4 A = Av[b];
                        const float qb = qv[b];
                        const float X0 = fmaf(fc0, A.x, A.y), X1 = fmaf(fc1, A.x, A.y), X2 = fmaf(fc2, A.x, A.y);
                        const float Y0 = fmaf(fr0, A.z, A.w), Y1 = fmaf(fr1, A.z, A.w), Y2 = fmaf(fr2, A.z, A.w);
                        const float xl0 = fminf(X0, X1), xh0 = fmaxf(X0, X1), xl1 = fminf(X1, X2), xh1 = fmaxf(X1, X2);
                        const float yl0 = fminf(Y0, Y1), yh0 = fmaxf(Y0, Y1), yl1 = fminf(Y1, Y2), yh1 = fmaxf(Y1, Y2);
                        a00 = fmaf(fmaxf(fminf(xh0, yh0) - fmaxf(xl0, yl0), 0.0f), qb, a00);
                        a01 = fmaf(fmaxf(fminf(xh1, yh0) - fmaxf(xl1, yl0), 0.0f), qb, a01);
                        a10 = fmaf(fmaxf(fminf(xh0, yh1) - fmaxf(xl0, yl1), 0.0f), qb, a10);
                        a11 = fmaf(fmaxf(fminf(xh1, yh1) - fmaxf(xl1, yl1), 0.0f), qb, a11);
                    }
                }
            }
            float *__restrict__ fo = fout + sd.img0 + (long long)i * L * L;
            fo[(long long)r * L + c] = a00;
            if (c + 1 < L) fo[(long long)r * L + c + 1] = a01;
            if (r + 1 < L) {
                fo[(long long)(r + 1) * L + c] = a10;
                if (c + 1 < L) fo[(long long)(r + 1) * L + c + 1] = a11;
            }
        }
        if (partials != nullptr) {
            double sq = 0.0;
            if (any) {
                sq = (double)a00 * (double)a00;
                if (c + 1 < L) sq += (double)a01 * (double)a01;
                if (r + 1 < L) {
                    sq += (double)a10 * (double)a10;
                    if (c + 1 < L) sq += (double)a11 * (double)a11;
                }
            }
            const double tot = block_sum_256(sq, sh);
            if (threadIdx.x == 0) partials[sd.gp0 + (long long)i * sd.nbp + tcy * nt + tcx] = tot;
        }
    }
    work_end(st);
}

void launch_backproject(const Batch &b, const Stage &st, const float *q, float *f, double *partials,
                        hipStream_t strm) {
    if (st.total == 0) return;
    k_backproject<<<st.grid, kBlock, 0, strm>>>(b, st, q, f, partials);
}

}  // namespace tnlm
