/*
 * FP64 CPU oracle of the temporal non-local means (TNLM) 4DCT reconstruction
 * (Tian, Jia, Dong, Lou, Jiang, "Low-dose 4DCT reconstruction via temporal
 * non-local means", arXiv:1009.1351).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously-correct
 * reference against which the HIP path is checked. It shares no code, header,
 * table or constant generator with the HIP library, and the product path never
 * links, loads or calls it. Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark use it.
 *
 * Everything is double precision and written as plain loops in the order of the
 * paper's equations and algorithm boxes:
 *   geometry and Siddon projector ....... §2.1 (P_i), §3 (Siddon, fan-beam arc)
 *   matched back-projector P^T .......... Eq. 4 and the CGLS box of §2.2
 *   FBP initial image ................... TNLM algorithm box, step 1
 *   CGLS data step ...................... §2.2, CGLS algorithm box, P_n = S^-1/2 P
 *   gradient step (M1 = 0) .............. Eq. 4
 *   adaptive patch weights .............. Eq. 8 (form of Eq. 3), §2.3 window
 *   Gauss-Jacobi sweep, positivity ...... Eq. 7, Gauss-Jacobi box, TNLM box step 5
 *   outer loop .......................... TNLM algorithm box
 *   cost ................................ Eq. 1 with Eq. 2
 *
 * Readings of points the paper leaves open (each one is listed with its
 * reason in the design notes of the repository):
 *   - patch distance = plain sum of squared differences over the d x d patch
 *     (Eqs. 3 and 8 write the squared norm);
 *   - the candidate set of Eq. 8 is the W x W window around x (§2.3) truncated
 *     to the image, centre included, normalised over that set;
 *   - patch pixels outside the image take the nearest edge pixel's value;
 *   - weights are computed with the window-minimum distance subtracted before
 *     the exponential (identical to Eq. 8 in exact arithmetic);
 *   - phases form a ring (f_0 = f_N, f_{N+1} = f_1, §2.1); for N = 1 the
 *     neighbour of a phase is itself, for N = 2 both neighbours are the other;
 *   - Gauss-Jacobi = every phase updates from sweep m, weights frozen from g;
 *   - CGLS stops early for a phase (u unchanged from then on) when
 *     ||P_n^T r||^2 or ||P_n s||^2 is zero;
 *   - "until convergence" = relative L2 update of the whole phase stack below
 *     a tolerance, or a fixed iteration count when the tolerance is 0;
 *   - the FBP is the textbook equiangular fan-beam FBP (ramp filter, full
 *     360-degree scan) over the union of all phases' views.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    int32_t n_phases, L;
    double pixel_mm;
    int32_t n_views, n_bins;
    double sad_mm, sdd_mm, dgamma_rad, det_offset_bins;
    const double *view_angles; /* [N][V], radians */
} orc_geom;

typedef struct {
    int32_t patch, window;
    double h, mu_hat, beta;
    int32_t m1_cgls, m2_jacobi, max_outer;
    double tol_rel_update;
    const double *guide; /* NULL: weights from g^(k); else fixed weights from this [N][L][L] stack (Eq. 3) */
} orc_params;

/* ------------------------------------------------------------------------- */
/* Geometry: source on a circle of radius SAD, equiangular arc detector.      */
/* ------------------------------------------------------------------------- */
static void ray_of(const orc_geom *g, int i, int v, int b, double *sx, double *sy, double *ux,
                   double *uy) {
    double th = g->view_angles[(size_t)i * g->n_views + v];
    double gam = ((double)b - 0.5 * (g->n_bins - 1) + g->det_offset_bins) * g->dgamma_rad;
    *sx = g->sad_mm * cos(th);
    *sy = g->sad_mm * sin(th);
    *ux = cos(th + M_PI + gam);
    *uy = sin(th + M_PI + gam);
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/*
 * Siddon's method: the ray p(t) = s + t u (t in mm) meets the vertical grid
 * lines x = X0 + k D and horizontal lines y = Y0 + k D (k = 0..L) at
 * parametric values t; between two consecutive crossings inside the image
 * square the ray lies in exactly one pixel, found from the segment midpoint,
 * and the segment length is the system-matrix entry. Returns the number of
 * (pixel, length) pairs written (zero-length segments are dropped).
 */
static int siddon_trace(const orc_geom *g, double sx, double sy, double ux, double uy, int *pix,
                        double *len, double *tbuf) {
    const int L = g->L;
    const double D = g->pixel_mm, S = D * L, X0 = -0.5 * S, Y0 = -0.5 * S;
    double tmin = -INFINITY, tmax = INFINITY;
    if (fabs(ux) > 1e-15) {
        double a = (X0 - sx) / ux, b = (X0 + S - sx) / ux;
        tmin = fmax(tmin, fmin(a, b));
        tmax = fmin(tmax, fmax(a, b));
    } else if (!(sx > X0 && sx < X0 + S)) {
        return 0;
    }
    if (fabs(uy) > 1e-15) {
        double a = (Y0 - sy) / uy, b = (Y0 + S - sy) / uy;
        tmin = fmax(tmin, fmin(a, b));
        tmax = fmin(tmax, fmax(a, b));
    } else if (!(sy > Y0 && sy < Y0 + S)) {
        return 0;
    }
    if (!(tmax > tmin)) return 0;
    int nt = 0;
    tbuf[nt++] = tmin;
    tbuf[nt++] = tmax;
    if (fabs(ux) > 1e-15)
        for (int k = 0; k <= L; k++) {
            double t = (X0 + k * D - sx) / ux;
            if (t > tmin && t < tmax) tbuf[nt++] = t;
        }
    if (fabs(uy) > 1e-15)
        for (int k = 0; k <= L; k++) {
            double t = (Y0 + k * D - sy) / uy;
            if (t > tmin && t < tmax) tbuf[nt++] = t;
        }
    qsort(tbuf, (size_t)nt, sizeof(double), cmp_double);
    int ns = 0;
    for (int k = 0; k + 1 < nt; k++) {
        double l = tbuf[k + 1] - tbuf[k];
        if (!(l > 0.0)) continue;
        double tm = 0.5 * (tbuf[k] + tbuf[k + 1]);
        int c = (int)floor((sx + tm * ux - X0) / D);
        int r = (int)floor((sy + tm * uy - Y0) / D);
        if (c < 0 || c >= L || r < 0 || r >= L) continue;
        pix[ns] = r * L + c;
        len[ns] = l;
        ns++;
    }
    return ns;
}

/* q_i = P_i f_i for every phase. f: [N][L][L], q: [N][V][B]. */
void orc_project(const orc_geom *g, const double *f, double *q) {
    const int N = g->n_phases, V = g->n_views, B = g->n_bins, L = g->L;
#pragma omp parallel
    {
        int *pix = (int *)malloc(sizeof(int) * (size_t)(4 * L + 8));
        double *len = (double *)malloc(sizeof(double) * (size_t)(4 * L + 8));
        double *tb = (double *)malloc(sizeof(double) * (size_t)(4 * L + 8));
#pragma omp for schedule(dynamic)
        for (int iv = 0; iv < N * V; iv++) {
            int i = iv / V, v = iv % V;
            const double *fi = f + (size_t)i * L * L;
            for (int b = 0; b < B; b++) {
                double sx, sy, ux, uy;
                ray_of(g, i, v, b, &sx, &sy, &ux, &uy);
                int ns = siddon_trace(g, sx, sy, ux, uy, pix, len, tb);
                double acc = 0.0;
                for (int k = 0; k < ns; k++) acc += len[k] * fi[pix[k]];
                q[((size_t)i * V + v) * B + b] = acc;
            }
        }
        free(pix);
        free(len);
        free(tb);
    }
}

/* f_i = P_i^T q_i: the same (ray, pixel, length) triples, accumulated into pixels. */
void orc_backproject(const orc_geom *g, const double *q, double *f) {
    const int N = g->n_phases, V = g->n_views, B = g->n_bins, L = g->L;
    memset(f, 0, sizeof(double) * (size_t)N * L * L);
#pragma omp parallel
    {
        int *pix = (int *)malloc(sizeof(int) * (size_t)(4 * L + 8));
        double *len = (double *)malloc(sizeof(double) * (size_t)(4 * L + 8));
        double *tb = (double *)malloc(sizeof(double) * (size_t)(4 * L + 8));
#pragma omp for schedule(dynamic)
        for (int i = 0; i < N; i++) {
            double *fi = f + (size_t)i * L * L;
            for (int v = 0; v < V; v++)
                for (int b = 0; b < B; b++) {
                    double sx, sy, ux, uy;
                    ray_of(g, i, v, b, &sx, &sy, &ux, &uy);
                    int ns = siddon_trace(g, sx, sy, ux, uy, pix, len, tb);
                    double qv = q[((size_t)i * V + v) * B + b];
                    for (int k = 0; k < ns; k++) fi[pix[k]] += len[k] * qv;
                }
        }
        free(pix);
        free(len);
        free(tb);
    }
}

/* Writes the Siddon (pixel, length) list of one ray; returns its length. */
int orc_trace_ray(const orc_geom *g, int i, int v, int b, int32_t *pix, double *len) {
    double sx, sy, ux, uy;
    ray_of(g, i, v, b, &sx, &sy, &ux, &uy);
    int *p = (int *)malloc(sizeof(int) * (size_t)(4 * g->L + 8));
    double *tb = (double *)malloc(sizeof(double) * (size_t)(4 * g->L + 8));
    int ns = siddon_trace(g, sx, sy, ux, uy, p, len, tb);
    for (int k = 0; k < ns; k++) pix[k] = p[k];
    free(p);
    free(tb);
    return ns;
}

/* ------------------------------------------------------------------------- */
/* FBP (TNLM box step 1): equiangular fan-beam filtered back-projection.       */
/* Kak & Slaney, Principles of Computerized Tomographic Imaging, ch. 3:        */
/*   R'(g)  = R(g) * SAD * cos(g)                                             */
/*   Q(n a) = a * sum_k R'(k a) h(n - k),  h(0) = 1/(8 a^2),                   */
/*            h(odd n) = -1 / (2 pi^2 sin^2(n a)),  h(even n != 0) = 0         */
/*   f(x)   = dbeta * sum_views Q(gamma'(x)) / |x - s|^2   (linear interp.)    */
/* ------------------------------------------------------------------------- */
void orc_fbp(const orc_geom *g, const double *y, double *f, int all_phases) {
    const int N = g->n_phases, V = g->n_views, B = g->n_bins, L = g->L;
    const double a = g->dgamma_rad, D = g->pixel_mm, S = D * L;
    double *Q = (double *)malloc(sizeof(double) * (size_t)N * V * B);
    double *hk = (double *)malloc(sizeof(double) * (size_t)(2 * B));
    for (int n = -(B - 1); n <= B - 1; n++) {
        double v;
        if (n == 0) v = 1.0 / (8.0 * a * a);
        else if (n % 2 == 0) v = 0.0;
        else {
            double s = sin(n * a);
            v = -1.0 / (2.0 * M_PI * M_PI * s * s);
        }
        hk[n + B - 1] = v;
    }
#pragma omp parallel for schedule(static)
    for (int iv = 0; iv < N * V; iv++) {
        const double *row = y + (size_t)iv * B;
        double *out = Q + (size_t)iv * B;
        for (int n = 0; n < B; n++) {
            double acc = 0.0;
            for (int k = 0; k < B; k++) {
                double gk = ((double)k - 0.5 * (B - 1) + g->det_offset_bins) * a;
                acc += row[k] * g->sad_mm * cos(gk) * hk[n - k + B - 1];
            }
            out[n] = a * acc;
        }
    }
    int nout = all_phases ? 1 : N;
    int views_per_image = all_phases ? N * V : V;
    double dbeta = 2.0 * M_PI / views_per_image;
#pragma omp parallel for schedule(dynamic)
    for (int o = 0; o < nout * L; o++) {
        int img = o / L, r = o % L;
        for (int c = 0; c < L; c++) {
            double px = (c + 0.5) * D - 0.5 * S, py = (r + 0.5) * D - 0.5 * S;
            double acc = 0.0;
            for (int i = 0; i < N; i++) {
                if (!all_phases && i != img) continue;
                for (int v = 0; v < V; v++) {
                    double th = g->view_angles[(size_t)i * V + v];
                    double sx = g->sad_mm * cos(th), sy = g->sad_mm * sin(th);
                    double dx = px - sx, dy = py - sy;
                    double gam = atan2(dy, dx) - (th + M_PI);
                    gam = remainder(gam, 2.0 * M_PI);
                    double u = gam / a + 0.5 * (B - 1) - g->det_offset_bins;
                    int b0 = (int)floor(u);
                    double fr = u - b0;
                    const double *Qr = Q + ((size_t)i * V + v) * B;
                    double qv = 0.0;
                    if (b0 >= 0 && b0 < B) qv += (1.0 - fr) * Qr[b0];
                    if (b0 + 1 >= 0 && b0 + 1 < B) qv += fr * Qr[b0 + 1];
                    acc += qv / (dx * dx + dy * dy);
                }
            }
            f[((size_t)img * L + r) * L + c] = dbeta * acc;
        }
    }
    if (all_phases)
        for (int i = 1; i < N; i++) memcpy(f + (size_t)i * L * L, f, sizeof(double) * (size_t)L * L);
    free(Q);
    free(hk);
}

/* ------------------------------------------------------------------------- */
/* Data step (§2.2): CGLS on P_n = S^-1/2 P, y_n = S^-1/2 y, from u0 = f.      */
/* w = diag(S^-1) (inverse variances). M1 = 0 selects the gradient step Eq. 4. */
/* ------------------------------------------------------------------------- */
static double dot(const double *a, const double *b, size_t n) {
    double s = 0.0;
    for (size_t k = 0; k < n; k++) s += a[k] * b[k];
    return s;
}

static orc_geom one_phase(const orc_geom *g, int i) {
    orc_geom h = *g;
    h.n_phases = 1;
    h.view_angles = g->view_angles + (size_t)i * g->n_views;
    return h;
}

void orc_cgls(const orc_geom *g, const double *y, const double *w, const double *f, int m1,
              double beta, double *gout) {
    const int N = g->n_phases, L = g->L;
    const size_t ni = (size_t)L * L, ns = (size_t)g->n_views * g->n_bins;
    /* phases are independent problems: one thread per phase (the projector
       calls inside run single-threaded in that case) */
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < N; i++) {
    double *u = (double *)malloc(sizeof(double) * ni), *s = (double *)malloc(sizeof(double) * ni);
    double *t = (double *)malloc(sizeof(double) * ni);
    double *r = (double *)malloc(sizeof(double) * ns), *q = (double *)malloc(sizeof(double) * ns);
    double *tmp = (double *)malloc(sizeof(double) * ns);
    {
        orc_geom gi = one_phase(g, i);
        const double *yi = y + i * ns, *wi = w + i * ns;
        memcpy(u, f + i * ni, sizeof(double) * ni);
        if (m1 == 0) { /* Eq. 4: g = f - (1/beta) P^T S^-1 (P f - y) */
            orc_project(&gi, u, q);
            for (size_t k = 0; k < ns; k++) tmp[k] = wi[k] * (q[k] - yi[k]);
            orc_backproject(&gi, tmp, t);
            for (size_t k = 0; k < ni; k++) u[k] -= t[k] / beta;
            memcpy(gout + i * ni, u, sizeof(double) * ni);
            goto done;
        }
        /* r0 = y_n - P_n u0 ; s0 = P_n^T r0 */
        orc_project(&gi, u, q);
        for (size_t k = 0; k < ns; k++) r[k] = sqrt(wi[k]) * (yi[k] - q[k]);
        for (size_t k = 0; k < ns; k++) tmp[k] = sqrt(wi[k]) * r[k];
        orc_backproject(&gi, tmp, s);
        double gamma = dot(s, s, ni); /* ||P_n^T r^(m)||^2 */
        for (int m = 0; m < m1; m++) {
            if (!(gamma > 1e-300)) break;
            /* step 1: a = ||P_n^T r||^2 / ||P_n s||^2 */
            orc_project(&gi, s, q);
            for (size_t k = 0; k < ns; k++) q[k] *= sqrt(wi[k]);
            double qq = dot(q, q, ns);
            if (!(qq > 0.0)) break;
            double a = gamma / qq;
            /* steps 2, 3 */
            for (size_t k = 0; k < ni; k++) u[k] += a * s[k];
            for (size_t k = 0; k < ns; k++) r[k] -= a * q[k];
            /* steps 4, 5: b = ||P_n^T r^(m+1)||^2 / ||P_n^T r^(m)||^2, s = P_n^T r + b s */
            for (size_t k = 0; k < ns; k++) tmp[k] = sqrt(wi[k]) * r[k];
            orc_backproject(&gi, tmp, t);
            double gnew = dot(t, t, ni);
            double bcoef = gnew / gamma;
            for (size_t k = 0; k < ni; k++) s[k] = t[k] + bcoef * s[k];
            gamma = gnew;
        }
        memcpy(gout + i * ni, u, sizeof(double) * ni); /* step 6: g = u^(M1) */
    }
    done:
    free(u); free(s); free(t); free(r); free(q); free(tmp);
    }
}

/* ------------------------------------------------------------------------- */
/* Patch weights, Eq. 8 with the §2.3 search window.                         */
/* ------------------------------------------------------------------------- */
static inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* SSD between the d x d patch of image a around (r, c) and of image b around (r2, c2). */
static double patch_ssd(const double *a, const double *b, int L, int d, int r, int c, int r2, int c2) {
    int s = d / 2;
    double acc = 0.0;
    for (int py = -s; py <= s; py++)
        for (int px = -s; px <= s; px++) {
            double e = a[clampi(r + py, 0, L - 1) * L + clampi(c + px, 0, L - 1)] -
                       b[clampi(r2 + py, 0, L - 1) * L + clampi(c2 + px, 0, L - 1)];
            acc += e * e;
        }
    return acc;
}

/*
 * Normalised weights w(x, y) for one pixel x = (r, c) of image gi against
 * image gj over the W x W window; out-of-image candidates get NaN. Also
 * returns the distances if dist != NULL. W*W entries each, row-major in (dy, dx).
 */
void orc_weights(int L, int d, int W, double h, const double *gi, const double *gj, int r, int c,
                 double *wout, double *dist) {
    int R = W / 2;
    double m = INFINITY;
    for (int dy = -R; dy <= R; dy++)
        for (int dx = -R; dx <= R; dx++) {
            int k = (dy + R) * W + (dx + R), r2 = r + dy, c2 = c + dx;
            if (r2 < 0 || r2 >= L || c2 < 0 || c2 >= L) {
                wout[k] = NAN;
                if (dist) dist[k] = NAN;
                continue;
            }
            double D = patch_ssd(gi, gj, L, d, r, c, r2, c2);
            wout[k] = D;
            if (dist) dist[k] = D;
            if (D < m) m = D;
        }
    double Z = 0.0;
    for (int k = 0; k < W * W; k++)
        if (!isnan(wout[k])) {
            wout[k] = exp(-(wout[k] - m) / (h * h));
            Z += wout[k];
        }
    for (int k = 0; k < W * W; k++)
        if (!isnan(wout[k])) wout[k] /= Z;
}

/* sum_y w_{i,j}(x, y) value_j(y) for one pixel. */
static double weighted_neighbour(int L, int d, int W, double h, const double *gi, const double *gj,
                                 const double *vj, int r, int c, double *wbuf) {
    orc_weights(L, d, W, h, gi, gj, r, c, wbuf, NULL);
    int R = W / 2;
    double acc = 0.0;
    for (int dy = -R; dy <= R; dy++)
        for (int dx = -R; dx <= R; dx++) {
            double wk = wbuf[(dy + R) * W + (dx + R)];
            if (isnan(wk)) continue;
            acc += wk * vj[(r + dy) * L + (c + dx)];
        }
    return acc;
}

/*
 * One Gauss-Jacobi sweep (Eq. 7 / Gauss-Jacobi box, step 1):
 *   out_i(x) = g_i(x)/(1+mu) + mu/(2mu+2) [ sum_y w_{i,i-1} value_{i-1}(y)
 *                                         + sum_y w_{i,i+1} value_{i+1}(y) ]
 * with weights from the guide stack (Eq. 8). clamp != 0 applies max(., 0)
 * (TNLM box, step 5). Stacks are [N][L][L].
 */
void orc_regularize(int N, int L, int d, int W, double h, double mu_hat, const double *guide,
                    const double *value, const double *g, double *out, int clamp) {
    const size_t ni = (size_t)L * L;
#pragma omp parallel
    {
        double *wbuf = (double *)malloc(sizeof(double) * (size_t)W * W);
#pragma omp for schedule(dynamic)
        for (int ir = 0; ir < N * L; ir++) {
            int i = ir / L, r = ir % L;
            int im = (i - 1 + N) % N, ip = (i + 1) % N;
            for (int c = 0; c < L; c++) {
                double am = weighted_neighbour(L, d, W, h, guide + i * ni, guide + im * ni,
                                               value + im * ni, r, c, wbuf);
                double ap = weighted_neighbour(L, d, W, h, guide + i * ni, guide + ip * ni,
                                               value + ip * ni, r, c, wbuf);
                double u = g[i * ni + r * L + c] / (1.0 + mu_hat) + mu_hat / (2.0 * mu_hat + 2.0) * (am + ap);
                if (clamp && u < 0.0) u = 0.0;
                out[i * ni + r * L + c] = u;
            }
        }
        free(wbuf);
    }
}

/* M2 Gauss-Jacobi sweeps from u0 = g with weights frozen from the guide
 * stack (g itself when guide is NULL); then f = max(u, 0). */
void orc_gauss_jacobi(int N, int L, int d, int W, double h, double mu_hat, int m2, const double *g,
                      const double *guide, double *f) {
    const size_t n = (size_t)N * L * L;
    double *u = (double *)malloc(sizeof(double) * n), *un = (double *)malloc(sizeof(double) * n);
    memcpy(u, g, sizeof(double) * n);
    for (int m = 0; m < m2; m++) {
        orc_regularize(N, L, d, W, h, mu_hat, guide ? guide : g, u, g, un, 0);
        memcpy(u, un, sizeof(double) * n);
    }
    for (size_t k = 0; k < n; k++) f[k] = u[k] > 0.0 ? u[k] : 0.0;
    free(u);
    free(un);
}

/* ------------------------------------------------------------------------- */
/* Outer loop (TNLM algorithm box).                                           */
/* ------------------------------------------------------------------------- */
/* One outer iteration in place: f <- f^(k) from f^(k-1). Returns the relative update. */
double orc_step(const orc_geom *g, const orc_params *p, const double *y, const double *w, double *f) {
    const size_t n = (size_t)g->n_phases * g->L * g->L;
    double *gk = (double *)malloc(sizeof(double) * n), *fn = (double *)malloc(sizeof(double) * n);
    orc_cgls(g, y, w, f, p->m1_cgls, p->beta, gk);                                   /* step 2 */
    orc_gauss_jacobi(g->n_phases, g->L, p->patch, p->window, p->h, p->mu_hat, p->m2_jacobi, gk, p->guide,
                     fn); /* steps 3-5 */
    double dd = 0.0, nn = 0.0;
    for (size_t k = 0; k < n; k++) {
        dd += (fn[k] - f[k]) * (fn[k] - f[k]);
        nn += fn[k] * fn[k];
    }
    memcpy(f, fn, sizeof(double) * n);
    free(gk);
    free(fn);
    return sqrt(dd) / fmax(sqrt(nn), 1e-30);
}

/*
 * Full solve. init_fbp != 0: f^(0) = FBP of all phases' views (box step 1);
 * otherwise f holds the caller's f^(0). Runs max_outer iterations, stopping
 * early once the relative update drops below tol (tol > 0). Returns the number
 * of iterations done; *rel_out receives the last relative update and
 * rel_hist (nullable, max_outer entries) every one of them.
 */
int orc_solve(const orc_geom *g, const orc_params *p, const double *y, const double *w, double *f,
              int init_fbp, double *rel_out, double *rel_hist) {
    if (init_fbp) orc_fbp(g, y, f, 1);
    double rel = 0.0;
    int k = 0;
    while (k < p->max_outer) {
        rel = orc_step(g, p, y, w, f);
        if (rel_hist) rel_hist[k] = rel;
        k++;
        if (p->tol_rel_update > 0.0 && rel < p->tol_rel_update) break;
    }
    if (rel_out) *rel_out = rel;
    return k;
}

/*
 * Cost of Eq. 1 (with J of Eq. 2): data = sum_i (P f_i - y_i)^T S^-1 (P f_i - y_i),
 * reg = sum_i [J(f_i, f_{i-1}) + J(f_i, f_{i+1})] with weights from the guide
 * stack. The total cost is data + (mu/2) reg with mu = mu_hat * beta.
 */
void orc_cost(const orc_geom *g, const orc_params *p, const double *y, const double *w, const double *f,
              const double *guide, double *data_out, double *reg_out) {
    const int N = g->n_phases, L = g->L, W = p->window, R = W / 2;
    const size_t ni = (size_t)L * L, ns = (size_t)N * g->n_views * g->n_bins;
    double *q = (double *)malloc(sizeof(double) * ns);
    orc_project(g, f, q);
    double data = 0.0;
    for (size_t k = 0; k < ns; k++) data += w[k] * (q[k] - y[k]) * (q[k] - y[k]);
    double reg = 0.0;
#pragma omp parallel reduction(+ : reg)
    {
        double *wb = (double *)malloc(sizeof(double) * (size_t)W * W);
#pragma omp for schedule(dynamic)
        for (int ir = 0; ir < N * L; ir++) {
            int i = ir / L, r = ir % L;
            int nb[2] = {(i - 1 + N) % N, (i + 1) % N};
            for (int c = 0; c < L; c++)
                for (int t = 0; t < 2; t++) {
                    int j = nb[t];
                    orc_weights(L, p->patch, W, p->h, guide + i * ni, guide + j * ni, r, c, wb, NULL);
                    double fx = f[i * ni + r * L + c];
                    for (int dy = -R; dy <= R; dy++)
                        for (int dx = -R; dx <= R; dx++) {
                            double wk = wb[(dy + R) * W + (dx + R)];
                            if (isnan(wk)) continue;
                            double e = fx - f[j * ni + (r + dy) * L + (c + dx)];
                            reg += e * e * wk;
                        }
                }
        }
        free(wb);
    }
    free(q);
    *data_out = data;
    *reg_out = reg;
}

/*
 * beta of the splitting (Eq. 4): an estimate of the largest eigenvalue of
 * P_i^T S^-1 P_i (the Lipschitz constant of the data-term gradient / 2), by
 * power iteration from the all-ones image; the maximum over phases.
 */
double orc_power_beta(const orc_geom *g, const double *w, int iters) {
    const int N = g->n_phases, L = g->L;
    const size_t ni = (size_t)L * L, ns = (size_t)g->n_views * g->n_bins;
    double best = 0.0;
    double *x = (double *)malloc(sizeof(double) * ni), *z = (double *)malloc(sizeof(double) * ni);
    double *q = (double *)malloc(sizeof(double) * ns);
    for (int i = 0; i < N; i++) {
        orc_geom gi = one_phase(g, i);
        for (size_t k = 0; k < ni; k++) x[k] = 1.0 / sqrt((double)ni);
        double lam = 0.0;
        for (int it = 0; it < iters; it++) {
            orc_project(&gi, x, q);
            for (size_t k = 0; k < ns; k++) q[k] *= w[i * ns + k];
            orc_backproject(&gi, q, z);
            double nz = sqrt(dot(z, z, ni));
            lam = nz;
            if (!(nz > 0.0)) break;
            for (size_t k = 0; k < ni; k++) x[k] = z[k] / nz;
        }
        if (lam > best) best = lam;
    }
    free(x); free(z); free(q);
    return best;
}
