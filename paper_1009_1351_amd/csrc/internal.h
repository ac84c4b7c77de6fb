// Internal declarations shared by the library's HIP translation units.
//
// Every kernel works on a *batch* of slices described by a slice table: each
// slice has its own image side L, views V, bins B and offsets into the batch's
// contiguous arrays. A kernel launch covers the blocks of all slices; blocks
// find their slice by binary search in a per-stage prefix table and loop over
// work items (persistent grid-stride loop). A single slice is a batch of one.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tnlm.h"

namespace tnlm {

struct SliceDesc {
    int N, L, V, B;
    float D;         // pixel size (mm)
    float X0;        // -L*D/2: left/bottom edge of the image square
    float dgamma;    // angular bin pitch
    float ucenter;   // (B-1)/2 - det_offset: bin coordinate of the central ray
    long long ray0;  // first ray of this slice in the ray tables ([N][V][B])
    long long view0; // first view in the view table ([N][V])
    long long img0;  // first element in image-shaped arrays ([N][L][L])
    long long sino0; // first element in sinogram-shaped arrays ([N][V][B])
    long long pimg0; // first element in the projector's padded image copies ([N][L][L + 2])
    int gp0, qp0, rp0;   // first partial slot in gpart / qpart / relpart
    int nbp, npp, nrb;   // partial slots per phase (transpose, projector) and per slice (regulariser)
    int hf0, cw0;        // first entry of this slice's FBP filter taps (2B-1) and cosine weights (B)
    int phase0;          // first global phase index of this slice
};

// Per-stage block prefix: blocks of slice s are [pre[s], pre[s+1]).
struct Stage {
    const int *pre;   // device [ns + 1]
    const int *xb;    // device [9]: work items [xb[x], xb[x+1]) go to XCD x
    int total;        // pre[ns]
    int grid;         // persistent grid size
    int cu_runs = 0;  // 1: blocks sharing a CU take consecutive work items
    int *queue = nullptr;   // device [9] (nullable): per-XCD item counters and a finished-block count
    int prefetch = 0; // 1: a block asks for its next item while it works on the current one
};

struct Batch {
    int ns = 0;
    const SliceDesc *sl = nullptr;   // device [ns]
    const float4 *rt0 = nullptr;     // rays: (Ax, Bx, Ay, By), T_x(k) = fma(k, Ax, Bx)
    const float4 *vt = nullptr;      // views: (sx, sy, cos th, sin th)
    const int4 *vo = nullptr;        // views: (bx, by, flags, 0), sign changes of Ax / Ay over the bins
    const int *skip = nullptr;       // device [ns] per-slice stop flags (nullable: run all)
};

struct RegParams {
    int patch, window;
    float h, mu_hat;
};

// Tables the host fills at set-up (stage prefixes, slice descriptors, view
// tables) are never written by a kernel. Read through the constant address
// space, a wave-uniform index loads them with scalar loads into scalar
// registers.
template <class T>
__device__ __forceinline__ T load_const(const T *p, long long i) {
    static_assert(sizeof(T) % 4 == 0, "tables are made of 4-byte words");
    using cword = const __attribute__((address_space(4))) int;
    cword *src = (cword *)(p + i);
    T out;
    int *dst = reinterpret_cast<int *>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
    return out;
}

// Work items currently in a stage (the device table, which the host may
// re-cut between launches; Stage::total is the count at set-up).
__device__ __forceinline__ int stage_total(const Stage &st) { return load_const(st.xb, 8); }

// Block index -> (slice, local block). Block-uniform.
__device__ __forceinline__ int find_slice(const int *pre, int ns, int gb) {
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (load_const(pre, mid) <= gb) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Persistent loop order: the 8 XCDs receive consecutive hardware block ids in
// turn; each XCD gets a contiguous range of work items, so that the blocks
// sharing an XCD (and its L2) work on the same slices and phases. The ranges
// are cut on the host to equal estimated cost (slices of a batch differ in
// size and view count), not to equal item counts. The tables live in device
// memory, so the host can re-cut them between launches (when slices of a
// batch have converged) without changing the launch itself.
__device__ __forceinline__ void xcd_range(const Stage &st, int &first, int &stride, int &count) {
    const int nx = 8;
    const int g = (int)gridDim.x;
    if (g < nx) {   // fewer blocks than XCDs: plain grid-stride order
        first = (int)blockIdx.x;
        stride = g;
        count = load_const(st.xb, nx);
        return;
    }
    const int x = (int)blockIdx.x % nx;
    const int per_x = (g - x + nx - 1) / nx;          // blocks on this XCD
    int k = (int)blockIdx.x / nx;                      // rank within the XCD
    // the blocks of an XCD are spread over its 32 CUs in turn: on request,
    // give the blocks that share a CU (ranks j, j + 32, ...) consecutive work
    // items, whose rays overlap in that CU's L1 (projector pair)
    constexpr int kCUsPerXCD = 32;
    if (st.cu_runs && per_x % kCUsPerXCD == 0) k = (k % kCUsPerXCD) * (per_x / kCUsPerXCD) + k / kCUsPerXCD;
    first = load_const(st.xb, x) + k;
    stride = per_x;
    count = load_const(st.xb, x + 1);
}

// Work items of a stage for one block. With a queue, the blocks of XCD x
// take the items [xb[x], xb[x+1]) one at a time, in the order they ask, from
// a counter: the items an XCD works on at once stay consecutive for the whole
// launch (with a fixed grid-stride order, blocks drift apart over the many
// items each takes, until the XCD works on images from several phases and
// slices at once and its L2 no longer holds them). The last block to finish
// clears the counters for the next launch. Results do not depend on which
// block takes an item. Without a queue, the fixed order of xcd_range.
// Every thread of the block must call work_next and work_end.
// With st.prefetch, thread 0 asks for the item after the one it hands out at
// once, so that the counter's reply arrives while the block works on the
// current item; a block processes every item it obtains below the end, and
// the call that meets the end asks for nothing more. (Each block then holds
// two items, which widens the range an XCD's L2 serves at once: worth it for
// many short items, not for a few long ones.)
struct WorkIter {
    int cur, stride, end, x;
    int next;   // thread 0: the item already obtained for the next call (-1: none yet)
};

__device__ __forceinline__ WorkIter work_begin(const Stage &st) {
    WorkIter it;
    xcd_range(st, it.cur, it.stride, it.end);
    it.x = (int)blockIdx.x % 8;
    it.next = -1;
    return it;
}

__device__ __forceinline__ bool work_next(const Stage &st, WorkIter &it, int &gb, int *sh_item) {
    if (st.queue && gridDim.x >= 8) {
        if (threadIdx.x == 0) {
            const int base = load_const(st.xb, it.x);
            const int item = it.next >= 0 ? it.next : base + atomicAdd(st.queue + it.x, 1);
            *sh_item = item;
            if (st.prefetch) it.next = item < it.end ? base + atomicAdd(st.queue + it.x, 1) : it.end;
        }
        __syncthreads();
        gb = *sh_item;
        __syncthreads();   // read by every thread before the next item's grab
        return gb < it.end;
    }
    gb = it.cur;
    it.cur += it.stride;
    return gb < it.end;
}

__device__ __forceinline__ void work_end(const Stage &st) {
    if (!st.queue || gridDim.x < 8 || threadIdx.x != 0) return;
    __threadfence();
    if (atomicAdd(st.queue + 8, 1) == (int)gridDim.x - 1) {   // every block has finished taking items
        for (int k = 0; k < 9; ++k) st.queue[k] = 0;
        __threadfence();
    }
}

// ---- projector (proj.hip)
enum ProjMode { PROJ_PLAIN = 0, PROJ_RESID = 1, PROJ_SCALED = 2 };
int proj_blocks(const SliceDesc &s);
int bp_blocks(const SliceDesc &s);
int tr_blocks(const SliceDesc &s);
// fP, fTP: the image stack copied row-major and transposed per phase, each
// row padded with a zero column on either side ([N][L][L + 2] per slice at
// pimg0; the owner of the buffers clears the zero columns once)
void launch_transpose(const Batch &b, const Stage &st, const float *f, float *fP, float *fTP, hipStream_t strm);
// f, fT: the padded copies written by launch_transpose
void launch_project(const Batch &b, const Stage &st, int mode, const float *f, const float *fT, const float *y,
                    const float *sw, float *out, float *out2, double *partials, hipStream_t strm);
void launch_backproject(const Batch &b, const Stage &st, const float *q, float *f, double *partials,
                        hipStream_t strm);

// ---- CGLS vector work (cgls.hip)
struct CglsBufs {
    float *u, *s, *t;           // image-shaped
    float *r, *q, *rw, *sw;     // sinogram-shaped
    double *gpart[2];           // partial ||P^T r||^2 (ping-pong)
    double *qpart;              // partial ||P s||^2
    int *stop;                  // [M1+1][total phases] CGLS stop flags
    int nphase;                 // total phases in the batch
};
int vec_blocks(const SliceDesc &s);   // per phase
void launch_sqrt(const float *w, float *sw, size_t n, hipStream_t st);
void launch_copy(const float *src, float *dst, size_t n, hipStream_t st);
void launch_copy_skip(const Batch &b, const Stage &st, bool image, const float *src, float *dst, hipStream_t strm);
void launch_cgls_update(const Batch &b, const Stage &st, CglsBufs &cb, int m, int gsel, hipStream_t strm);
void launch_cgls_direction(const Batch &b, const Stage &st, CglsBufs &cb, int m, int gold, int gnew,
                           hipStream_t strm);
void launch_weighted_resid(const Batch &b, const Stage &st, const float *q, const float *y, const float *w,
                           float *out, hipStream_t strm);
void launch_gradient_step(const Batch &b, const Stage &st, const float *f, const float *bp, float inv_beta,
                          float *gout, hipStream_t strm);
void launch_finalize(const Batch &b, const double *relpart, float tol, float *hist, int *counter, int *done,
                     const int *nonfinite, int max_outer, hipStream_t strm);
void launch_check_finite(const float *a, size_t n, int *flag, hipStream_t st);
void launch_fill_int(int *a, int n, int v, hipStream_t st);
int launch_wsq_sum(const float *q, const float *y, const float *w, size_t n, double *part, hipStream_t st);
// partials [2 * blocks] of ||a - b||^2 and ||a||^2; *bad += non-finite entries (set it to 0 first)
int launch_diff_sq(const float *a, const float *b, size_t n, double *part, int *bad, hipStream_t st);

// ---- TNLM regulariser (tnlm_reg.hip)
int reg_blocks(const SliceDesc &s, int patch, int rows_per_lane);
// regularisation term of Eq. 1 (one slice); returns the number of partial sums in part
int launch_reg_cost(int N, int L, int patch, int window, float h, const float *guide, const float *f, double *part,
                    int max_blocks, hipStream_t strm);
bool reg_supported(int patch, int window);
void launch_regularize(const Batch &b, const Stage &st, const RegParams &p, int rows_per_lane,
                       const float *guide, const float *value, const float *g, float *out, int clamp,
                       double *relpart, int *nonfinite, hipStream_t strm);

// ---- regulariser with BF16 MFMA patch distances (tnlm_reg_mfma.hip)
int reg_mfma_blocks(const SliceDesc &s);
bool reg_mfma_supported(int patch, int window);
// symmetric reuse of §2.3 (ssd_mode FP32_SYMMETRIC): one pass over the
// unordered phase pairs, then the per-pixel combination (two launches)
bool reg_sym_supported(int patch, int window);
int reg_sym_planes(int patch, int window);   // image-shaped planes of reverse partial sums
int reg_sym_rows_per_lane();
void launch_regularize_sym(const Batch &b, const Stage &st, const RegParams &p, const float *guide,
                           const float *value, const float *g, float *out, int clamp, double *relpart,
                           int *nonfinite, float2 *fwd, float2 *part, size_t nimg, hipStream_t strm);
void launch_regularize_mfma(const Batch &b, const Stage &st, const RegParams &p, const float *guide,
                            const float *value, const float *g, float *out, int clamp, double *relpart,
                            int *nonfinite, hipStream_t strm);

// ---- FBP (fbp.hip)
void launch_fbp(const Batch &b, const Stage &filt, const Stage &bp, const float *y, const float *hfilt,
                const float *cosw, float *Q, float *f, int all_phases, hipStream_t strm);
int fbp_bp_blocks(const SliceDesc &s, int all_phases);

}  // namespace tnlm
