// Internal declarations shared by the library's HIP translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>
#include <algorithm>

#include "../../include/tnlm.h"

namespace tnlm {

// Per-slice device geometry: everything a projector kernel needs.
struct DevGeom {
    int N, L, V, B;
    float D;         // pixel size (mm)
    float X0;        // -L*D/2: left/bottom edge of the image square
    float dgamma;    // angular bin pitch
    float ucenter;   // (B-1)/2 - det_offset: bin coordinate of the central ray
    const float4 *rt0;   // [N][V][B] plane tables (Ax, Bx, Ay, By): T_x(k) = fma(k, Ax, Bx)
    const float4 *rt1;   // [N][V][B] (ox, oy, ux, uy): ray point nearest the centre, direction
    const float4 *vt;    // [N][V] (sx, sy, cos th, sin th)
};

struct RegShape {
    int N, L, patch, window;
    float h, mu_hat;
};

// ---- projector (proj.hip)
enum ProjMode { PROJ_PLAIN = 0, PROJ_RESID = 1, PROJ_SCALED = 2 };
int proj_blocks_per_phase(const DevGeom &g);
void launch_project(const DevGeom &g, int mode, const float *f, const float *y, const float *sw, float *out,
                    float *out2, double *partials, const int *skip, hipStream_t st);
int bp_blocks_per_phase(const DevGeom &g);
void launch_backproject(const DevGeom &g, const float *q, float *f, double *partials, const int *skip,
                        hipStream_t st);

// ---- CGLS vector work (cgls.hip)
struct CglsBufs {
    float *u, *s, *t;        // [N][L][L]
    float *r, *q, *rw, *sw;  // [N][V][B]
    double *gpart[2];        // [N][nbp]: partial ||P^T r||^2 (ping-pong)
    double *qpart;           // [N][npp]: partial ||P s||^2
    int *stop;               // [M1+1][N] CGLS stop flags
    int nbp, npp;
};
void launch_sqrt(const float *w, float *sw, size_t n, hipStream_t st);
void launch_copy(const float *src, float *dst, size_t n, const int *skip, hipStream_t st);
void launch_cgls_update(const DevGeom &g, CglsBufs &b, int m, int gsel, const int *skip, hipStream_t st);
void launch_cgls_direction(const DevGeom &g, CglsBufs &b, int m, int gsel_old, int gsel_new, const int *skip,
                           hipStream_t st);
void launch_gradient_step(const DevGeom &g, const float *f, const float *bp, float inv_beta, float *gout,
                          const int *skip, hipStream_t st);
void launch_weighted_resid(const DevGeom &g, const float *q, const float *y, const float *w, float *out,
                           const int *skip, hipStream_t st);
void launch_finalize(const double *partials, int nblocks, float tol, float *hist, int *counter, int *done,
                     int *nonfinite, int max_outer, const int *skip, hipStream_t st);
void launch_check_finite(const float *a, size_t n, int *flag, hipStream_t st);

// ---- TNLM regulariser (tnlm_reg.hip)
int reg_blocks(const RegShape &s);
bool reg_supported(int patch, int window);
void launch_regularize(const RegShape &s, const float *guide, const float *value, const float *g, float *out,
                       int clamp, double *relpart, int *nonfinite, const int *skip, hipStream_t st);

// ---- FBP (fbp.hip)
void launch_fbp(const DevGeom &g, const float *y, const float *hfilt, const float *cosw, float *Q, float *f,
                int all_phases, float sad, hipStream_t st);

}  // namespace tnlm
