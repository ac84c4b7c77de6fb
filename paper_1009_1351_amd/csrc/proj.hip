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
// row, writes are coalesced); rows in which every ray of a wave is inside the
// image take an unmasked loop. Transpose: one lane
// per pixel, a deterministic gather over views and the pixel's candidate
// bins (no floating-point atomics). Both are persistent over the batch's
// ragged slice table.
#include "devutil.h"
#include "internal.h"

namespace tnlm {

__device__ __forceinline__ float plane_t(int k, float A, float B) { return fmaf((float)k, A, B); }

// Rays per lane (adjacent bins; the walk is written for any count). One:
// two rays per lane give each pass twice the arithmetic to cover the
// latency of its reads, but spread a wave's reads over twice the cache
// lines and raise the registers to 76 (6 waves per SIMD); measured slower.
constexpr int kProjRays = 1;
constexpr int kRaysPerBlock = kBlock * kProjRays;

int proj_blocks(const SliceDesc &s) { return s.N * s.V * ((s.B + kRaysPerBlock - 1) / kRaysPerBlock); }

// The walk reads zero-padded copies of the image stack: each row of L pixels
// is stored with one zero column on either side (row stride L + 2, pixel
// (r, c) at r (L + 2) + c + 1), so the cell just past a side of the image
// reads 0. Reads go through a buffer resource spanning one padded phase
// image: an offset outside it reads 0 without a memory access.
__device__ __forceinline__ int padded_stride(int L) { return L + 2; }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const float *fi, int L) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(fi), (short)0, L * padded_stride(L) * 4, 0x00020000);
}

__device__ __forceinline__ float image_at(__amdgpu_buffer_rsrc_t img, int byte_off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(img, byte_off, 0, 0));
}

// Cells c and c + dc of a row (byte offsets off and off + ox): two reads.
__device__ __forceinline__ float2 image_two(__amdgpu_buffer_rsrc_t img, int off, int ox) {
    return make_float2(image_at(img, off), image_at(img, off + ox));
}

__device__ __forceinline__ float cell_clip(float xl, float xh, float yl, float yh) {
    return fmaxf(fminf(xh, yh) - fmaxf(xl, yl), 0.0f);
}

// Offset that the image's buffer resource turns into a read of 0 without a
// memory access (beyond the padded L x (L + 2) image for every L the engine
// accepts, also after the steps a lane that takes no part adds to it).
constexpr int kNoCell = 0x40000000;

// State of one ray's walk between passes. Column c holds the ray at the
// start of a pass (its upper x plane txh = T_x(fkx) lies beyond the pass's
// lower y plane tyl); rowoff is the byte offset of column -1 of the pass's
// row in the padded image; v1, v2 are the cells (r, c) and (r, c + dc) read
// ahead for the pass. pin, pout and pside are the passes of the ray's entry
// row, of its exit row (with margin) and of the row in which it leaves
// through the side it runs towards (L if it leaves through the far row edge).
struct Walk {
    int c, dc, rowoff, ox, oy, pin, pout, pside;
    float fkx, fky, dcf, drf, txh, tyl, tin, acc;
    float v1, v2;             // cells c and c + dc of the pass's row
    bool hit, dead;
};

// Entry and exit of one ray (plane tables A: x planes in .x/.y, y planes in
// .z/.w, and ray points O, both in the wave's frame).
__device__ __forceinline__ void walk_setup(Walk &w, const float4 A, const float4 O, bool valid, int L, float X0,
                                           float invD) {
    int pin = L, pout = -1, pside = L, c = 0, dc = 1, dr = 1, hc = 1, hr = 1;
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
            // pass in which the walk meets the side plane it runs towards (the
            // first pass whose upper y plane is not below that plane's T, the
            // comparison the walk makes), or L if it leaves through the far row
            // edge first: estimated from the point on that plane, then settled
            // on the plane values
            const float tse = plane_t(dc > 0 ? L : 0, A.x, A.y);
            int rs = (int)floorf((fmaf(tse, O.w, O.y) - X0) * invD);
            rs = min(max(rs, 0), L - 1);
            int ps = max(dr > 0 ? rs : L - 1 - rs, pin);
            auto ty_up = [&](int p) { return plane_t((dr > 0 ? p : L - 1 - p) + hr, A.z, A.w); };
            while (ps > pin && tse <= ty_up(ps - 1)) --ps;
            while (ps < L && !(tse <= ty_up(ps))) ++ps;
            pside = ps;
        }
    }
    w.c = c;
    w.dc = dc;
    w.ox = 4 * dc;
    w.dcf = (float)dc;
    w.drf = (float)dr;
    w.fkx = (float)(c + hc);
    w.txh = plane_t(c + hc, A.x, A.y);
    w.tin = tin;
    w.acc = 0.0f;
    w.hit = hit;
    w.dead = !hit;
    w.pin = pin;
    w.pout = pout;
    w.pside = pside;
    (void)hr;
}

// Row-dependent part of the state at the wave's first pass p0.
__device__ __forceinline__ void walk_start(Walk &w, const float4 A, int L, int p0) {
    const int dr = w.drf > 0.0f ? 1 : -1, hr = dr > 0 ? 1 : 0;
    const int r0 = dr > 0 ? p0 : L - 1 - p0;
    const int LP = padded_stride(L);
    w.oy = 4 * dr * LP;
    w.rowoff = 4 * r0 * LP;
    w.fky = (float)(r0 + hr);
    w.tyl = plane_t(r0 + 1 - hr, A.z, A.w);
}

__device__ __forceinline__ void walk_load(Walk &w, __amdgpu_buffer_rsrc_t img, bool live) {
    const int o1 = live ? w.rowoff + 4 * w.c + 4 : kNoCell;
    const float2 v = image_two(img, o1, w.ox);
    w.v1 = v.x;
    w.v2 = v.y;
}

// One pass of one ray with the masks that rows before its entry row and
// after its side exit need. At the start of a pass a live ray's column c
// holds it and the column's upper x plane lies beyond the row's lower y
// plane (txh > tyl), so the clip of (r, c) is non-negative and that of
// (r, c + dc) has max(txh, tyl) = txh: both are the transpose kernel's clips
// without its clamp. The lower x plane of column c is at most tyl in every
// row but the entry row, where it is tin or at most tin = tyl, so
// max(x_lo, tyl) = max(tin, tyl) throughout. A ray that is not live reads 0.
__device__ __forceinline__ void masked_pass(Walk &w, int p, const float4 A, __amdgpu_buffer_rsrc_t img, int L) {
    const bool live = !w.dead && p >= w.pin;
    const float tyh = fmaf(w.fky, A.z, A.w);
    const float txn = fmaf(w.fkx + w.dcf, A.x, A.y);
    const float l1 = fminf(w.txh, tyh) - fmaxf(w.tin, w.tyl);
    const float l2 = fminf(txn, tyh) - w.txh;
    const bool cross = live && w.txh <= tyh;   // reaches the next column in this row
    const bool in2 = (unsigned)(w.c + w.dc) < (unsigned)L;
    const bool take2 = cross && in2;
    w.acc = fmaf(l1, w.v1, w.acc);
    w.acc = fmaf(take2 ? l2 : 0.0f, w.v2, w.acc);
    w.dead = w.dead || (cross && !in2);   // left the image through a side
    w.c = take2 ? w.c + w.dc : w.c;
    w.fkx = take2 ? w.fkx + w.dcf : w.fkx;
    w.txh = take2 ? txn : w.txh;
    while (take2 && w.txh <= tyh) {   // a further column in the same row
        if ((unsigned)(w.c + w.dc) >= (unsigned)L) {
            w.dead = true;
            break;
        }
        const float tx3 = fmaf(w.fkx + w.dcf, A.x, A.y);
        w.acc = fmaf(cell_clip(w.txh, tx3, w.tyl, tyh), image_at(img, w.rowoff + 4 * (w.c + w.dc) + 4), w.acc);
        w.c += w.dc;
        w.fkx += w.dcf;
        w.txh = tx3;
    }
    w.tyl = tyh;
    w.fky += w.drf;
    w.rowoff += w.oy;
    walk_load(w, img, !w.dead && p + 1 >= w.pin);   // next row's cells, in flight during the next pass
}

// Passes [pa, pb) of both rays with masks.
__device__ __forceinline__ void walk_masked(Walk (&w)[kProjRays], int pa, int pb, const float4 (&A)[kProjRays],
                                            __amdgpu_buffer_rsrc_t img, int L) {
    if (pa >= pb) return;
#pragma unroll
    for (int j = 0; j < kProjRays; ++j) walk_load(w[j], img, !w[j].dead && pa >= w[j].pin);
    for (int p = pa; p < pb; ++p) {
#pragma unroll
        for (int j = 0; j < kProjRays; ++j) masked_pass(w[j], p, A[j], img, L);
    }
}

// Unmasked stretch of one ray: the carried state between its passes.
struct Steady {
    float lo, edge;
    float va1, va2, vb1, vb2;   // cells of alternate passes (no load's destination is copied: a copy waits)
    int o1, ox, oy, oxy;
};

__device__ __forceinline__ void steady_begin(Steady &s, Walk &w, __amdgpu_buffer_rsrc_t img, int L) {
    s.lo = fmaxf(w.tin, w.tyl);
    // the column ahead lies past the side once dc * fkx >= dc * (plane index
    // of that side): the current column is the last one or already outside
    s.edge = w.dcf * (w.dc > 0 ? (float)L : 0.0f);
    s.ox = w.hit ? w.ox : 0;
    s.oy = w.hit ? w.oy : 0;
    s.oxy = s.ox + s.oy;
    if (!w.hit) w.txh = INFINITY;   // never crosses a column: sp = tyh, l2 = 0, and it reads 0
    s.o1 = w.hit ? w.rowoff + 4 * w.c + 4 : kNoCell;   // cell c of the pass
    const float2 v = image_two(img, s.o1, s.ox);
    s.va1 = v.x;
    s.va2 = v.y;
    s.vb1 = s.vb2 = 0.0f;
}

// One unmasked pass of one ray. The arithmetic of each entry is that of
// masked_pass for a live ray:
//   * lo = max(tin, tyl) at the stretch's first pass and tyl after it (tin <
//     tyl once the entry row is behind);
//   * the length in column c + dc is min(txn, tyh) - min(txh, tyh): the
//     masked pass's min(txn, tyh) - txh when the ray reaches that column in
//     this row (txh <= tyh), and exactly 0 when it does not (txn >= txh >
//     tyh), so no mask is needed;
//   * a ray leaving through a side in the stretch's last pass reads the zero
//     padding as its cell (r, c + dc) and adds 0.
// The next pass's cells (cv1, cv2 are this pass's; nv1, nv2 receive the
// next's) are requested as soon as their column is known: it follows from
// this pass's crossing test alone unless the ray crosses two columns in this
// row (then they are requested again). The column is tracked through the
// read offset o1 and the plane index fkx only.
__device__ __forceinline__ void steady_pass(Steady &s, Walk &w, const float4 A, __amdgpu_buffer_rsrc_t img,
                                            const float &cv1, const float &cv2, float &nv1, float &nv2) {
    const float tyh = fmaf(w.fky, A.z, A.w);
    const bool cross = w.txh <= tyh;
    int o1n = s.o1 + (cross ? s.oxy : s.oy);   // next row; next column too when the ray reaches it
    {
        const float2 nv = image_two(img, o1n, s.ox);
        nv1 = nv.x;
        nv2 = nv.y;
    }
    const float fkn = w.fkx + w.dcf;
    const float txn = fmaf(fkn, A.x, A.y);
    const float sp = fminf(w.txh, tyh);
    const float l1 = sp - s.lo;
    const float l2 = fminf(txn, tyh) - sp;
    w.acc = fmaf(l1, cv1, w.acc);
    w.acc = fmaf(l2, cv2, w.acc);
    w.fkx = cross ? fkn : w.fkx;
    w.txh = cross ? txn : w.txh;
    if (cross && w.txh <= tyh) {   // a further column in the same row (rare)
        int oc = o1n - s.oy;   // the column entered, in this pass's row
        while (w.txh <= tyh) {
            if (w.dcf * w.fkx >= s.edge) {   // the next column is past the side: step onto it and stop
                w.fkx += w.dcf;             // (this is the ray's side-exit pass, the stretch's last)
                break;
            }
            const float tx3 = fmaf(w.fkx + w.dcf, A.x, A.y);
            w.acc = fmaf(cell_clip(w.txh, tx3, s.lo, tyh), image_at(img, oc + s.ox), w.acc);
            oc += s.ox;
            w.fkx += w.dcf;
            w.txh = tx3;
        }
        o1n = oc + s.oy;
        const float2 rv = image_two(img, o1n, s.ox);
        nv1 = rv.x;
        nv2 = rv.y;
    }
    s.lo = tyh;
    w.fky += w.drf;
    s.o1 = o1n;
}

// Passes [pa, pb] in which every ray of the wave that meets the image is
// inside it: at or after its entry row and at or before the row in which it
// leaves through a side. Rays that miss the image read at kNoCell with
// ox = oy = 0 and add 0.
__device__ __forceinline__ void walk_steady(Walk (&w)[kProjRays], int pa, int pb, const float4 (&A)[kProjRays],
                                            __amdgpu_buffer_rsrc_t img, int L) {
    if (pa > pb) return;
    Steady s[kProjRays];
#pragma unroll
    for (int j = 0; j < kProjRays; ++j) steady_begin(s[j], w[j], img, L);
    int p = pa;
    for (; p < pb; p += 2) {
#pragma unroll
        for (int j = 0; j < kProjRays; ++j) steady_pass(s[j], w[j], A[j], img, s[j].va1, s[j].va2, s[j].vb1, s[j].vb2);
#pragma unroll
        for (int j = 0; j < kProjRays; ++j) steady_pass(s[j], w[j], A[j], img, s[j].vb1, s[j].vb2, s[j].va1, s[j].va2);
    }
    if (p == pb) {
#pragma unroll
        for (int j = 0; j < kProjRays; ++j) steady_pass(s[j], w[j], A[j], img, s[j].va1, s[j].va2, s[j].vb1, s[j].vb2);
    }
    // back to the masked walk's state: column from the plane index; a ray
    // whose column is past a side left the image in the stretch's last pass
#pragma unroll
    for (int j = 0; j < kProjRays; ++j) {
        w[j].tyl = s[j].lo;
        if (w[j].hit) {
            w[j].rowoff += (pb - pa + 1) * w[j].oy;
            w[j].c = (int)w[j].fkx - (w[j].dc > 0 ? 1 : 0);
            if ((unsigned)w[j].c >= (unsigned)L) w[j].dead = true;
        }
    }
}

// Row-synchronous walk of one wave's rays over one phase image (L x L,
// padded). The plane tables and ray points come in the wave's frame, in
// which every ray of the wave crosses about one column per row or fewer.
// Pass p visits image row p counted along the rays' row direction for all
// rays at once, so the lanes of a wave read neighbouring cells of one row
// (two per ray: the current column and the next) rather than drifting apart
// by their different numbers of column crossings. The length of each cell is
// the clip of the transpose kernel and cells are added in the order the ray
// meets them (a ray that reaches the next column exactly at the row's upper
// plane enters it with length 0 first), so the sum is bitwise that of a walk
// crossing one grid line at a time. The wave runs from the first entry row
// to the last exit row of its rays, in three stretches: masked passes up to
// the last entry row of the wave, unmasked passes while every ray is inside
// the image, masked passes after the first side exit; a ray crossing two
// columns in one row takes the rare inner loop.
// Must be called by all lanes of the wave; rays with valid = false add nothing.
__device__ __forceinline__ void walk_rows(const float4 (&A)[kProjRays], const float4 (&O)[kProjRays],
                                          const bool (&valid)[kProjRays], __amdgpu_buffer_rsrc_t img, int L,
                                          float X0, float invD, float (&acc)[kProjRays]) {
    Walk w[kProjRays];
    int p0 = L, p1 = -1, pa = 0, pb = L;
#pragma unroll
    for (int j = 0; j < kProjRays; ++j) {
        walk_setup(w[j], A[j], O[j], valid[j], L, X0, invD);
        p0 = min(p0, w[j].pin);
        p1 = max(p1, w[j].pout);
        if (w[j].hit) {
            pa = max(pa, w[j].pin);
            pb = min(pb, w[j].pside);
        }
    }
    for (int m = 32; m > 0; m >>= 1) {
        p0 = min(p0, __shfl_xor(p0, m, 64));
        p1 = max(p1, __shfl_xor(p1, m, 64));
        pa = max(pa, __shfl_xor(pa, m, 64));
        pb = min(pb, __shfl_xor(pb, m, 64));
    }
    p0 = wave_uniform(p0);
    p1 = wave_uniform(p1);
    pa = max(wave_uniform(pa), p0);   // first pass of the unmasked stretch
    pb = min(wave_uniform(pb), p1);   // its last pass
#pragma unroll
    for (int j = 0; j < kProjRays; ++j) walk_start(w[j], A[j], L, p0);
    if (pa <= pb) {
        walk_masked(w, p0, pa, A, img, L);
        walk_steady(w, pa, pb, A, img, L);
        walk_masked(w, pb + 1, p1 + 1, A, img, L);
    } else {
        walk_masked(w, p0, p1 + 1, A, img, L);
    }
#pragma unroll
    for (int j = 0; j < kProjRays; ++j) acc[j] = w[j].acc;
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

// One pass over the image stack writes both padded copies the projector
// reads: row-major and transposed, each row with a zero column on either side
// (the zero columns are cleared once when the buffers are allocated and never
// written).
__global__ __launch_bounds__(kBlock) void k_transpose(Batch bt, Stage st, const float *__restrict__ f,
                                                      float *__restrict__ fP, float *__restrict__ fTP) {
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
        const int LP = L + 2;
        const float *__restrict__ src = f + sd.img0 + (long long)i * L * L;
        float *__restrict__ dst = fP + sd.pimg0 + (long long)i * L * LP;
        float *__restrict__ dstT = fTP + sd.pimg0 + (long long)i * L * LP;
        for (int k = 0; k < kTr; k += kBlock / kTr) {
            const int r = by * kTr + ty + k, c = bx * kTr + tx;
            if (r < L && c < L) {
                const float v = src[r * L + c];
                tile[ty + k][tx] = v;
                dst[r * LP + c + 1] = v;
            }
        }
        __syncthreads();
        for (int k = 0; k < kTr; k += kBlock / kTr) {
            const int c = bx * kTr + ty + k, r = by * kTr + tx;
            if (r < L && c < L) dstT[c * LP + r + 1] = tile[tx][ty + k];
        }
        __syncthreads();
    }
}

void launch_transpose(const Batch &b, const Stage &st, const float *f, float *fP, float *fTP, hipStream_t strm) {
    if (st.total == 0) return;
    k_transpose<<<st.grid, kBlock, 0, strm>>>(b, st, f, fP, fTP);
}

template <int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_project(Batch bt, Stage st, const float *__restrict__ f,
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
        const int b0 = bx * kRaysPerBlock + kProjRays * threadIdx.x;   // the lane's rays: b0, b0 + 1
        const long long ray0 = ((long long)i * sd.V + v) * sd.B + b0;   // within the slice
        const int L = sd.L;
        float4 A[kProjRays], O[kProjRays];
        bool valid[kProjRays];
        int nval = 0, nxmaj = 0;
#pragma unroll
        for (int j = 0; j < kProjRays; ++j) {
            valid[j] = b0 + j < sd.B;
            A[j] = make_float4(1.0f, 0.0f, 1.0f, 0.0f);
            if (valid[j]) A[j] = bt.rt0[sd.ray0 + ray0 + j];
            nval += __popcll(__ballot(valid[j]));
            nxmaj += __popcll(__ballot(valid[j] && fabsf(A[j].x) < fabsf(A[j].z)));
        }
        // the wave walks the transposed image, axes exchanged, when most of
        // its rays cross columns faster than rows
        const bool tr = wave_uniform(2 * nxmaj > nval ? 1 : 0) != 0;
        if (tr) {
#pragma unroll
            for (int j = 0; j < kProjRays; ++j) A[j] = make_float4(A[j].z, A[j].w, A[j].x, A[j].y);
        }
        // a point of each ray and its direction, for the walk's estimates of
        // its entry and exit cells (settled afterwards on the plane values):
        // A.x = D / u_x and A.y = (X0 - o_x) / u_x, so u_x = D / A.x and
        // o_x = X0 - A.y u_x (likewise in y), to a few ulp
#pragma unroll
        for (int j = 0; j < kProjRays; ++j) {
            const float ux = sd.D * __builtin_amdgcn_rcpf(A[j].x), uy = sd.D * __builtin_amdgcn_rcpf(A[j].z);
            O[j] = make_float4(fmaf(-A[j].y, ux, sd.X0), fmaf(-A[j].w, uy, sd.X0), ux, uy);
        }
        const __amdgpu_buffer_rsrc_t img = image_rsrc((tr ? fT : f) + sd.pimg0 + (long long)i * L * (L + 2), L);
        float acc[kProjRays];
        walk_rows(A, O, valid, img, L, sd.X0, 1.0f / sd.D, acc);
        double part = 0.0;
#pragma unroll
        for (int j = 0; j < kProjRays; ++j) {
            if (!valid[j]) continue;
            const long long e = sd.sino0 + ray0 + j;
            if (MODE == PROJ_PLAIN) {
                out[e] = acc[j];
            } else if (MODE == PROJ_RESID) {   // r = sw (y - P u), rw = sw r
                const float w = sw[e];
                const float res = w * (y[e] - acc[j]);
                out[e] = res;
                out2[e] = w * res;
            } else {                           // q = sw P s, partial ||q||^2
                const float qv = sw[e] * acc[j];
                out[e] = qv;
                part += (double)qv * (double)qv;
            }
        }
        if (MODE == PROJ_SCALED) {
            const double tot = block_sum_256(part, sh);
            if (threadIdx.x == 0) partials[sd.qp0 + (long long)i * sd.npp + v * nbx + bx] = tot;
        }
    }    work_end(st);
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
// planes c, c+1, c+2 (and r, r+1, r+2) are evaluated once. With the signs
// known, the ray meets the 2 x 2 square in order: it enters at tin = max of
// the entry planes into the corner pixel on the entry sides, crosses the
// middle lines x1 and y1 (clamped into [tin, tout]), and leaves at tout =
// min of the exit planes from the opposite corner pixel; between min(x1, y1)
// and max(x1, y1) it is in the neighbour of the entry pixel across the line
// crossed first. Each length is the same difference of the same two plane
// values as the pixel's clip min(hi planes) - max(lo planes), and a pixel
// the ray misses gets +0, so the sums are those of the clips bit for bit
// (the forward walk's entries).
template <int R, int C>
__device__ __forceinline__ float &blk(float &a00, float &a01, float &a10, float &a11) {
    if constexpr (R == 0) return C == 0 ? a00 : a01;
    else return C == 0 ? a10 : a11;
}

template <bool XP, bool YP>
__device__ __forceinline__ void bp_block_ray(const float4 A, const float qb, float fc0, float fr0, float &a00,
                                             float &a01, float &a10, float &a11) {
    const float fc1 = fc0 + 1.0f, fc2 = fc0 + 2.0f, fr1 = fr0 + 1.0f, fr2 = fr0 + 2.0f;
    const float X0 = fmaf(fc0, A.x, A.y), X1 = fmaf(fc1, A.x, A.y), X2 = fmaf(fc2, A.x, A.y);
    const float Y0 = fmaf(fr0, A.z, A.w), Y1 = fmaf(fr1, A.z, A.w), Y2 = fmaf(fr2, A.z, A.w);
    const float tin = fmaxf(XP ? X0 : X2, YP ? Y0 : Y2);
    // max(min(exit planes), tin), which is tin when the ray misses the square:
    // the median of the three, since each entry plane lies at or before its
    // exit plane and so tin is at most the larger exit plane
    const float tout = __builtin_amdgcn_fmed3f(XP ? X2 : X0, YP ? Y2 : Y0, tin);
    const float x1 = __builtin_amdgcn_fmed3f(tin, X1, tout);
    const float y1 = __builtin_amdgcn_fmed3f(tin, Y1, tout);
    const float a = fminf(x1, y1), b = fmaxf(x1, y1);
    const float lmid = b - a;
    const bool xfirst = x1 < y1;
    constexpr int ci = XP ? 0 : 1, ri = YP ? 0 : 1;   // entry pixel
    float &ain = blk<ri, ci>(a00, a01, a10, a11);
    float &aout = blk<1 - ri, 1 - ci>(a00, a01, a10, a11);
    float &ax = blk<ri, 1 - ci>(a00, a01, a10, a11);   // across the x line from the entry pixel
    float &ay = blk<1 - ri, ci>(a00, a01, a10, a11);   // across the y line
    ain = fmaf(a - tin, qb, ain);
    ax = fmaf(xfirst ? lmid : 0.0f, qb, ax);
    ay = fmaf(xfirst ? 0.0f : lmid, qb, ay);
    aout = fmaf(tout - b, qb, aout);
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

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_backproject(Batch bt, Stage st, const float *__restrict__ q,
                                                        float *__restrict__ fout, double *__restrict__ partials) {
    __shared__ double sh[kBlock];
    __shared__ int sh_item;
    WorkIter it = work_begin(st);
    int gb;
    // a wave takes an 8 x 8 square of 2 x 2 blocks (16 x 16 pixels) of the
    // tile: its lanes' candidate bins then span the square's projected width,
    // less on average than a 32 x 8 strip's, so each 16-byte record load of
    // the wave touches fewer cache lines
    static_assert(kBpLanes == 16 && kBlock == 256, "four 8 x 8 squares of lanes per tile");
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int tx = (wv & 1) * 8 + (ln & 7), ty = (wv >> 1) * 8 + (ln >> 3);
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
    }    work_end(st);
}

void launch_backproject(const Batch &b, const Stage &st, const float *q, float *f, double *partials,
                        hipStream_t strm) {
    if (st.total == 0) return;
    k_backproject<<<st.grid, kBlock, 0, strm>>>(b, st, q, f, partials);
}



}  // namespace tnlm
