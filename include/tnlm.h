/*
 * tnlm.h -- C ABI of the MI355X (gfx950) TNLM 4DCT reconstruction library.
 *
 * Method: Tian, Jia, Dong, Lou, Jiang, "Low-dose 4DCT reconstruction via
 * temporal non-local means" (arXiv:1009.1351). All N respiratory phases f_i of
 * one CT slice are reconstructed jointly by minimising Eq. 1: a statistically
 * weighted data term (P_i f_i - y_i)^T S^-1 (P_i f_i - y_i) plus a temporal
 * non-local-means term coupling phase i with i-1 and i+1 on a ring of phases
 * (§2.1). The solver is the modified forward-backward splitting of §2.2:
 * per outer iteration, M1 CGLS steps on the whitened data term, new patch
 * weights from the CGLS output (Eq. 8, W x W window of §2.3), M2 Gauss-Jacobi
 * sweeps of Eq. 7, and a positivity clamp (TNLM algorithm box).
 *
 * Conventions shared by every entry point
 *   - Images: float32, [N][L][L] row-major; row index r along +y, column c
 *     along +x; pixel (r, c) centre = ((c+1/2) D - L D/2, (r+1/2) D - L D/2),
 *     D = pixel_mm.
 *   - Sinograms: float32, [N][V][B] (phase, view, bin), bins contiguous.
 *   - Geometry (§3): source at sad_mm * (cos th, sin th) for view angle th;
 *     equiangular arc detector; bin b has fan angle
 *     g_b = (b - (B-1)/2 + det_offset_bins) * dgamma_rad and its ray leaves
 *     the source with direction angle th + pi + g_b.
 *   - w: inverse variances S^-1 (diagonal), float32 [N][V][B], w >= 0.
 *   - Device pointers ("d_") are caller-owned HIP device memory on the device
 *     that was current at init; the library never frees or reallocates them.
 *     Host pointers are read during the call only.
 *   - All work is enqueued on the HIP stream given at init (a hipStream_t,
 *     passed as void*; NULL = the default stream). Calls marked "async" return
 *     before the GPU finishes; the others synchronise that stream once.
 *   - A context is used by one host thread at a time. Separate contexts on
 *     separate streams are independent.
 *   - Errors: every call returns a tnlm_status; 0 = success, < 0 = error
 *     (nothing is written on argument errors), > 0 = warning. A human-readable
 *     message of the last failure on the calling thread is returned by
 *     tnlm_last_error(). No C++ exception crosses this boundary.
 */
#ifndef TNLM_H
#define TNLM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TNLM_OK = 0,
    TNLM_E_INVALID_ARG = -1, /* bad scalar argument or null pointer          */
    TNLM_E_SHAPE = -2,       /* inconsistent sizes                           */
    TNLM_E_HIP = -3,         /* a HIP runtime call failed                    */
    TNLM_E_OOM = -4,         /* device allocation failed                     */
    TNLM_E_NONFINITE = -5,   /* NaN/Inf detected in inputs or iterates       */
    TNLM_W_NOT_CONVERGED = 1 /* max_outer reached before tol_rel_update      */
} tnlm_status;

enum { TNLM_INIT_FBP_ALL = 0, TNLM_INIT_USER = 1 };
/* How the regulariser forms the patch distances and weights of Eq. 8:
 *   TNLM_SSD_FP32            FP32 box sums, per-pixel running-minimum shift;
 *   TNLM_SSD_BF16_MFMA       cross terms on the BF16 matrix cores (patch 3, 5, 7;
 *                            window <= 15), compensated hi/lo split;
 *   TNLM_SSD_FP32_SYMMETRIC  the symmetric reuse of §2.3: each unordered pair of
 *                            neighbouring phases once, one distance and one
 *                            unshifted exponential per pair serving both
 *                            directions; a pixel whose weight sum underflows
 *                            (below 2^-60) is recomputed exactly. Same result
 *                            as TNLM_SSD_FP32 up to rounding; needs forward
 *                            and reverse partial sums (10 floats per image
 *                            element at window <= 17, 14 at 19). Window 21,
 *                            and window 19 with patch 3, need more than
 *                            64 KiB of LDS per block and are rejected with
 *                            TNLM_E_INVALID_ARG. */
enum { TNLM_SSD_FP32 = 0, TNLM_SSD_BF16_MFMA = 1, TNLM_SSD_FP32_SYMMETRIC = 2 };

typedef struct {
    int32_t n_phases;        /* N >= 1, phases on a ring (§2.1)               */
    int32_t L;               /* image side, 1 <= L <= 4096                     */
    double pixel_mm;         /* D > 0                                          */
    int32_t n_views;         /* V >= 1 per phase                               */
    int32_t n_bins;          /* B >= 1, B <= 4096                              */
    double sad_mm;           /* source to rotation centre (541.0 in §3)        */
    double sdd_mm;           /* source to detector (949.075 in §3)             */
    double dgamma_rad;       /* angular bin pitch                              */
    double det_offset_bins;  /* detector offset in bins (e.g. 0.25)            */
    const double *view_angles_rad; /* host [N][V]; copied at init           */
} tnlm_geometry;

typedef struct {
    int32_t patch;           /* d, odd, 3..9: patch side of Eq. 8             */
    int32_t window;          /* W, odd, 3..21, W <= L: search window (§2.3)    */
    float h;                 /* > 0: patch-distance scale of Eq. 8            */
    float mu_hat;            /* >= 0: mu / beta of Eq. 6-7                     */
    float beta;              /* > 0: FBS constant; used by M1 = 0 and the cost */
    int32_t m1_cgls;         /* M1 >= 0 CGLS steps (0 = gradient step, Eq. 4)  */
    int32_t m2_jacobi;       /* M2 >= 1 Gauss-Jacobi sweeps                    */
    int32_t max_outer;       /* >= 1 outer iterations (cap)                    */
    float tol_rel_update;    /* stop when ||F^k - F^k-1|| / ||F^k|| < tol; 0 = run max_outer */
    int32_t init;            /* TNLM_INIT_FBP_ALL or TNLM_INIT_USER            */
    int32_t ssd_mode;        /* TNLM_SSD_FP32, _BF16_MFMA or _FP32_SYMMETRIC   */
} tnlm_params;

typedef struct tnlm_ctx tnlm_ctx;

/*
 * Create a reconstruction context for one slice (geometry §3, parameters
 * §2.2-2.3). Builds the per-ray plane tables and allocates all scratch on
 * the current device. Validates: N >= 1, L >= 1, V >= 1, B >= 1, d and W odd
 * in range, W <= L, h > 0, mu_hat >= 0, beta > 0, M1 >= 0, M2 >= 1,
 * max_outer >= 1, tol >= 0. Returns TNLM_E_INVALID_ARG / TNLM_E_SHAPE /
 * TNLM_E_OOM / TNLM_E_HIP on failure (*out = NULL).
 */
tnlm_status tnlm_recon_init(tnlm_ctx **out, const tnlm_geometry *geom, const tnlm_params *params,
                            void *stream);
void tnlm_destroy(tnlm_ctx *ctx);

/*
 * One outer iteration of the TNLM algorithm box (steps 2-5), in place:
 * d_f holds f^(k-1) on entry and f^(k) on return. d_y, d_w: [N][V][B].
 * Async. The relative update is recorded on the device (tnlm_get_history).
 */
tnlm_status tnlm_step(tnlm_ctx *ctx, const float *d_y, const float *d_w, float *d_f);

/*
 * Full solve (TNLM algorithm box): f^(0) = FBP of all phases' views
 * (init = TNLM_INIT_FBP_ALL) or the caller's d_f (TNLM_INIT_USER); then outer
 * iterations until the relative update falls below tol_rel_update or
 * max_outer is reached. Synchronises once at the end. out_iters and
 * out_rel_update (host, nullable) receive the iteration count and the last
 * relative update. Returns TNLM_W_NOT_CONVERGED when tol > 0 was not reached,
 * TNLM_E_NONFINITE if an iterate became non-finite.
 */
tnlm_status tnlm_solve(tnlm_ctx *ctx, const float *d_y, const float *d_w, float *d_f, int32_t *out_iters,
                       float *out_rel_update);

/* Relative updates of the iterations done so far by tnlm_solve/tnlm_step
 * since init (host out[n]; synchronises). Returns the count in *out_n. */
tnlm_status tnlm_get_history(tnlm_ctx *ctx, float *out, int32_t n, int32_t *out_n);

/* q = P f (Siddon line integrals, §3), all phases. d_f [N][L][L] -> d_q [N][V][B]. Async. */
tnlm_status tnlm_project(tnlm_ctx *ctx, const float *d_f, float *d_q);

/* f = P^T q, the exact transpose of tnlm_project (Eq. 4, CGLS box). Async. */
tnlm_status tnlm_backproject(tnlm_ctx *ctx, const float *d_q, float *d_f);

/*
 * Filtered back-projection (TNLM box, step 1): equiangular fan-beam ramp
 * filter and distance-weighted back-projection over a full turn. all_phases
 * != 0: one image from the union of all N*V views, written to every phase
 * slot of d_f; 0: each phase from its own V views. Async.
 */
tnlm_status tnlm_fbp(tnlm_ctx *ctx, const float *d_y, float *d_f, int32_t all_phases);

/*
 * Data step of §2.2: M1 CGLS steps (CGLS box) on P_n = S^-1/2 P from
 * u0 = d_f, or the gradient step of Eq. 4 when M1 = 0; d_g <- g^(k).
 * d_f and d_g must not alias. Async.
 */
tnlm_status tnlm_data_step(tnlm_ctx *ctx, const float *d_y, const float *d_w, const float *d_f, float *d_g);

/*
 * One Gauss-Jacobi sweep of Eq. 7 with Eq. 8 weights:
 *   out_i(x) = g_i(x)/(1+mu) + mu/(2mu+2) * sum_{j=i-1,i+1} sum_y w_ij(x,y) value_j(y)
 * with w_ij computed from the guide stack (patch d, window W, h). clamp != 0
 * applies max(., 0). All stacks [N][L][L]; d_out must not alias the inputs.
 * For M2 = 1, guide = value = g. Async.
 */
tnlm_status tnlm_regularize(tnlm_ctx *ctx, const float *d_guide, const float *d_value, const float *d_g,
                            float *d_out, int32_t clamp);

/*
 * Kernel timing (tracing). While enabled, every kernel the context enqueues
 * is bracketed by a pair of HIP events recorded on the context's stream, and
 * tnlm_timing_read returns, per kernel kind, the summed event-to-event time
 * in milliseconds and the number of launches since the last read (it
 * synchronises the stream and resets the records). Enabling adds two event
 * records per launch; disable it outside measurements.
 */
enum {
    TNLM_KIND_PROJECT = 0,     /* forward projector (all modes)               */
    TNLM_KIND_BACKPROJECT = 1, /* transpose                                   */
    TNLM_KIND_REGULARIZE = 2,  /* weights + Gauss-Jacobi sweep                */
    TNLM_KIND_VECTOR = 3,      /* CGLS vector updates, copies                 */
    TNLM_KIND_FBP = 4,         /* filter + back-projection of the FBP         */
    TNLM_KIND_OTHER = 5,       /* reductions, checks                          */
    TNLM_KIND_COUNT = 6
};
tnlm_status tnlm_timing_enable(tnlm_ctx *ctx, int32_t enable);
tnlm_status tnlm_timing_read(tnlm_ctx *ctx, double *ms /* [TNLM_KIND_COUNT] */,
                             int32_t *launches /* [TNLM_KIND_COUNT] */);

/*
 * Autotuner of the regulariser tile: times the two supported tile heights
 * (4 or 8 output rows per lane, i.e. 16- or 32-row tiles) on the context's
 * first slice with synthetic images, requires their outputs to agree
 * bitwise, keeps the faster one for this context and appends the choice to a
 * JSON-lines cache (env TNLM_AUTOTUNE_CACHE, default
 * $HOME/.cache/tnlm_autotune.jsonl) keyed by (patch, window, L rounded up to
 * a power of two); later contexts of that class start from the cached
 * choice. A context (or batch) with FP32 distances whose class has no cached
 * choice runs this tuning once at creation; env TNLM_ROWS_PER_LANE (4 or 8)
 * forces a height and skips it. rows_per_lane (nullable) receives the choice,
 * ms (nullable, 2 floats) the kernel times of the 8- and 4-row candidates.
 * Synchronises.
 */
tnlm_status tnlm_autotune(tnlm_ctx *ctx, int32_t *rows_per_lane, float *ms);

/*
 * Batches of slices (many slices x N phases, uneven L, V, B). All slices
 * share the parameters; each has its own geometry (geoms[n_slices], host,
 * copied). One launch per stage covers every slice (blocks walk a ragged
 * slice table persistently); one outer iteration of the whole batch is
 * captured once into a hipGraph and replayed. Slices that reach
 * tol_rel_update stop (their work items are skipped) while the others go on.
 * The batch owns contiguous copies of y, w and f (inputs are copied in at
 * the start of tnlm_batch_solve, results copied out at the end).
 */
typedef struct tnlm_batch tnlm_batch;
tnlm_status tnlm_batch_init(tnlm_batch **out, int32_t n_slices, const tnlm_geometry *geoms,
                            const tnlm_params *params, void *stream);
void tnlm_batch_destroy(tnlm_batch *b);
/*
 * d_y, d_w, d_f: host arrays of n_slices device pointers (slice s: [N_s][V_s][B_s]
 * and [N_s][L_s][L_s]). out_iters, out_rel (host [n_slices], nullable) and
 * out_status (host [n_slices], nullable; per-slice TNLM_OK,
 * TNLM_W_NOT_CONVERGED or TNLM_E_NONFINITE). Returns the worst status.
 * Synchronises once at the end.
 */
tnlm_status tnlm_batch_solve(tnlm_batch *b, const float *const *d_y, const float *const *d_w, float *const *d_f,
                             int32_t *out_iters, float *out_rel, tnlm_status *out_status);
/*
 * As tnlm_batch_solve for the slices with active[s] != 0 (active: host
 * [n_slices]); the others take no part: their d_y, d_w, d_f are neither read
 * nor written (their pointers may be NULL), and they report 0 iterations and
 * TNLM_OK. With init = TNLM_INIT_USER a slice continues from d_f, so a solve
 * can resume a subset of a batch (the outer iteration's state is the image).
 */
tnlm_status tnlm_batch_solve_active(tnlm_batch *b, const float *const *d_y, const float *const *d_w,
                                   float *const *d_f, const int32_t *active, int32_t *out_iters, float *out_rel,
                                   tnlm_status *out_status);
tnlm_status tnlm_batch_timing_enable(tnlm_batch *b, int32_t enable);
tnlm_status tnlm_batch_timing_read(tnlm_batch *b, double *ms, int32_t *launches);

/*
 * Data term of Eq. 1 for the current iterate: out = sum_i (P_i f_i - y_i)^T S^-1
 * (P_i f_i - y_i) with S^-1 = diag(w) (double, host). Synchronises.
 */
tnlm_status tnlm_data_cost(tnlm_ctx *ctx, const float *d_y, const float *d_w, const float *d_f, double *out);

/*
 * Both terms of the cost of Eq. 1 for an image stack d_f ([N][L][L]):
 * out_data as tnlm_data_cost, out_reg = sum_i sum_{j = i-1, i+1} sum_x
 * sum_y w_ij(x, y) (f_i(x) - f_j(y))^2 over the search window inside the
 * image, with the normalised weights of Eq. 8 taken from d_guide ([N][L][L],
 * e.g. the data-step output g^(k)); the cost is out_data + mu_hat beta / 2
 * out_reg. Device arrays are caller-owned float32, results double on the
 * host. A diagnostic (direct patch sums, not the solve's kernels).
 * Synchronises.
 */
tnlm_status tnlm_cost(tnlm_ctx *ctx, const float *d_y, const float *d_w, const float *d_f, const float *d_guide,
                      double *out_data, double *out_reg);

/*
 * Fixed weights (Eq. 3 with a given image): from now on tnlm_step and
 * tnlm_solve take the patch weights of every Gauss-Jacobi sweep from d_guide
 * ([N][L][L] float32 device, caller-owned, read during those calls) instead
 * of from the data-step output g^(k); NULL restores the adaptive weights.
 * With the ground truth as guide this is the ideal-weight reference of the
 * method. Synchronises.
 */
tnlm_status tnlm_set_guide(tnlm_ctx *ctx, const float *d_guide);

/*
 * Relative change between two image stacks of the context's slice, as used by
 * the stop rule of the TNLM algorithm box: out = ||a - b|| / max(||a||, 1e-30)
 * over all phases (double sums, fixed order). Returns TNLM_E_NONFINITE if
 * either stack holds a NaN or infinity. Synchronises.
 */
tnlm_status tnlm_rel_change(tnlm_ctx *ctx, const float *d_a, const float *d_b, double *out);

/*
 * Learned warm start: an encoder-decoder network (4 levels with b, 2b, 4b, 8b
 * channels, two 3x3 convolutions + ReLU per level, 2x2 average pooling,
 * nearest 2x upsampling, skip concatenation, 1x1 head, residual to the input)
 * mapping the N per-phase FBP images of a slice ([n][N][H][W] float32, image
 * units) to an estimate of the converged TNLM images (same shape), used as
 * f^(0) of the TNLM algorithm box. BF16 weights and activations, FP32
 * accumulation, FP32 master weights and Adam moments; trained and run by the
 * library's own kernels. H and W must be multiples of 8. input_scale
 * multiplies the images before the network (e.g. 50 for attenuations ~0.02/mm).
 * Parameters: all weights [Cout][Cin][k][k] layer by layer, then all biases.
 */
typedef struct tnlm_cnn tnlm_cnn;
tnlm_status tnlm_cnn_create(tnlm_cnn **out, int32_t phases, int32_t base_channels, uint64_t seed, float input_scale,
                            void *stream);
void tnlm_cnn_destroy(tnlm_cnn *net);
int64_t tnlm_cnn_num_params(const tnlm_cnn *net);
tnlm_status tnlm_cnn_get_params(tnlm_cnn *net, float *host, int64_t n);
tnlm_status tnlm_cnn_set_params(tnlm_cnn *net, const float *host, int64_t n);
/* inference: d_out = network(d_in), both [n][N][H][W] float32 device. Async. */
tnlm_status tnlm_cnn_forward(tnlm_cnn *net, const float *d_in, float *d_out, int32_t n, int32_t H, int32_t W);
/* inference at a coarser grid: d_in is averaged over factor x factor blocks
 * (factor 1, 2, 4 or 8; H, W multiples of it), the network runs at
 * (H/factor, W/factor), and its output is upsampled bilinearly (pixel centres
 * aligned, edges clamped) into d_out [n][N][H][W]. Lets a network trained at
 * one pixel size serve slices at a finer one. Async. */
tnlm_status tnlm_cnn_forward_resampled(tnlm_cnn *net, const float *d_in, float *d_out, int32_t n, int32_t H,
                                       int32_t W, int32_t factor);
/* Bilinear upsampling of n images [n][h][w] -> [n][h*factor][w*factor]
 * (float32 device; output pixel X samples the input at (X + 1/2)/factor - 1/2,
 * clamped to the first and last pixel), e.g. a coarse-grid reconstruction as
 * the start of a fine one. Independent of any context; enqueued on `stream`
 * (hipStream_t as void*). Async. Errors: tnlm_cnn_last_error(). */
tnlm_status tnlm_image_upsample(const float *d_in, float *d_out, int32_t n, int32_t h, int32_t w, int32_t factor,
                                void *stream);
/* MSE loss (in input_scale units) and its gradient (host_grad nullable, num_params floats). Synchronises. */
tnlm_status tnlm_cnn_loss_grad(tnlm_cnn *net, const float *d_in, const float *d_target, int32_t n, int32_t H, int32_t W,
                               double *loss, float *host_grad, int64_t ngrad);
/* one Adam step (beta 0.9, 0.999, eps 1e-8) on the MSE loss; *loss = loss before the step. Synchronises. */
tnlm_status tnlm_cnn_train_step(tnlm_cnn *net, const float *d_in, const float *d_target, int32_t n, int32_t H,
                                int32_t W, float lr, double *loss);
/* checkpoint = parameters, Adam moments, step count; load validates shape and finiteness. */
tnlm_status tnlm_cnn_save(tnlm_cnn *net, const char *path);
tnlm_status tnlm_cnn_load(tnlm_cnn *net, const char *path);
const char *tnlm_cnn_last_error(void);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sweep of
 * tnlm_regularize for one slice of n_phases x L x L without a context. Same
 * arithmetic and the same bits as tnlm_regularize with (patch, window, h,
 * mu_hat) of a context of that slice. Stacks [n_phases][L][L] float32 on the
 * current device; d_out must not alias the inputs; enqueued on `stream`
 * (hipStream_t as void*, on the current device). Async.
 * No device or host allocation: the kernel's tables (slice descriptor and
 * work ranges) are written into a library-owned device array of 1 KiB per GPU,
 * held until the process ends. Every call on a GPU reuses that array, so
 * calls that may overlap on one GPU (different streams, or threads) race and
 * must be ordered by the caller. Sizes as tnlm_recon_init accepts them:
 * 1 <= L <= 4096, n_phases * L^2 <= 2^31 (else TNLM_E_SHAPE), window <= L,
 * patch odd in [3, 9], window odd in [3, 21].
 */
tnlm_status tnlm_regularize_noalloc(int32_t n_phases, int32_t L, int32_t patch, int32_t window, float h,
                                   float mu_hat, const float *d_guide, const float *d_value, const float *d_g,
                                   float *d_out, int32_t clamp, void *stream);

const char *tnlm_status_string(tnlm_status s);
const char *tnlm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TNLM_H */
