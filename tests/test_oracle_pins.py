"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, an invariant, a special case that reduces to a textbook routine, or an
independent brute force written here in NumPy with a different algorithm.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from synth.scan import ellipse_line_integrals
from synth.phantom import Ellipse, rasterize

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_geom(N=1, L=8, V=12, B=16, **kw):
    return synth.ScanGeometry(n_phases=N, L=L, n_views=V, n_bins=B, **kw)


def slab_interval(src, u, lo, hi):
    """Liang-Barsky clip of rays p = s + t u against the box [lo, hi]^2 (per axis arrays)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        tx0 = (lo[0] - src[..., 0]) / u[..., 0]
        tx1 = (hi[0] - src[..., 0]) / u[..., 0]
        ty0 = (lo[1] - src[..., 1]) / u[..., 1]
        ty1 = (hi[1] - src[..., 1]) / u[..., 1]
    tin = np.maximum(np.minimum(tx0, tx1), np.minimum(ty0, ty1))
    tout = np.minimum(np.maximum(tx0, tx1), np.maximum(ty0, ty1))
    return np.maximum(tout - tin, 0.0)


def dense_P_clip(geom):
    """Dense system matrix [N*V*B, N*L*L] from per-pixel box clipping (block-diagonal in phases)."""
    src, u = geom.rays()
    L, D, S = geom.L, geom.pixel_mm, geom.fov_mm
    N, V, B = geom.n_phases, geom.n_views, geom.n_bins
    A = np.zeros((N * V * B, N * L * L))
    for i in range(N):
        s = src[i].reshape(-1, 2)
        uu = u[i].reshape(-1, 2)
        for r in range(L):
            for c in range(L):
                lo = (-S / 2 + c * D, -S / 2 + r * D)
                hi = (lo[0] + D, lo[1] + D)
                A[i * V * B:(i + 1) * V * B, i * L * L + r * L + c] = slab_interval(s, uu, lo, hi)
    return A


def dense_P_oracle(orc, geom):
    G = orc.Geometry(geom)
    N, L = geom.n_phases, geom.L
    cols = []
    for k in range(N * L * L):
        e = np.zeros(N * L * L)
        e[k] = 1.0
        cols.append(orc.project(G, e.reshape(N, L, L)).ravel())
    return np.stack(cols, 1)


# --------------------------------------------------------------------- golden
def test_scanner_constants_golden():
    gold = json.load(open(os.path.join(GOLDEN, "scanner_constants.json")))
    from synth import geometry as sg
    assert sg.PAPER_DET_UNITS == gold["det_units"]
    assert sg.PAPER_DET_PITCH_MM == gold["det_pitch_mm"]
    assert sg.PAPER_SDD_MM == gold["sdd_mm"]
    assert sg.PAPER_SAD_MM == gold["sad_mm"]
    assert abs(sg.FAN_ANGLE_RAD - gold["derived"]["fan_angle_rad"]) < 1e-6
    fov_r = sg.PAPER_SAD_MM * math.sin(sg.FAN_ANGLE_RAD / 2)
    assert abs(fov_r - gold["derived"]["fov_radius_mm"]) < 0.01


# ------------------------------------------------------------------ projector
def test_P1_projection_of_ones_is_chord(orc):
    geom = small_geom(N=2, L=16, V=24, B=32)
    q = orc.project(orc.Geometry(geom), np.ones((2, 16, 16)))
    src, u = geom.rays()
    S = geom.fov_mm
    chord = slab_interval(src, u, (-S / 2, -S / 2), (S / 2, S / 2))
    np.testing.assert_allclose(q, chord, rtol=1e-12, atol=1e-9)
    assert (chord > 0).sum() > 0.5 * chord.size


def test_P2_siddon_equals_box_clipping_8x8(orc):
    geom = small_geom(N=2, L=8, V=12, B=16)
    A_clip = dense_P_clip(geom)
    A_orc = dense_P_oracle(orc, geom)
    np.testing.assert_allclose(A_orc, A_clip, rtol=0, atol=1e-11)
    assert np.count_nonzero(A_clip) > 500


def test_P3_siddon_converges_to_analytic_integral(orc):
    e = [Ellipse(20.0, -30.0, 120.0, 70.0, 0.4, 0.02)]
    errs = []
    for L in (32, 64, 128, 256):
        geom = small_geom(N=1, L=L, V=30, B=64)
        img = rasterize(e, L, supersample=8)[None]
        q = orc.project(orc.Geometry(geom), img)
        src, u = geom.rays()
        exact = ellipse_line_integrals(src, u, e)
        errs.append(np.linalg.norm(q - exact) / np.linalg.norm(exact))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.01


def test_P4_adjoint(orc):
    geom = small_geom(N=3, L=24, V=20, B=40)
    G = orc.Geometry(geom)
    rng = np.random.default_rng(4)
    f = rng.standard_normal((3, 24, 24))
    q = rng.standard_normal((3, 20, 40))
    lhs = np.dot(orc.project(G, f).ravel(), q.ravel())
    rhs = np.dot(f.ravel(), orc.backproject(G, q).ravel())
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0) * 10


# ----------------------------------------------------------------------- CGLS
def test_P5_cgls_is_krylov_minimiser(orc):
    geom = small_geom(N=1, L=6, V=10, B=12)
    G = orc.Geometry(geom)
    A = dense_P_oracle(orc, geom)
    rng = np.random.default_rng(5)
    w = rng.uniform(0.5, 2.0, size=A.shape[0])
    y = rng.uniform(0, 3, size=A.shape[0])
    u0 = rng.uniform(0, 0.02, size=A.shape[1])
    An = np.sqrt(w)[:, None] * A
    yn = np.sqrt(w) * y
    r0 = yn - An @ u0
    v = An.T @ r0
    K = []
    prev_res = np.linalg.norm(r0)
    for m in range(1, 6):
        K.append(v / np.linalg.norm(v))
        v = An.T @ (An @ K[-1])
        Km = np.stack(K, 1)
        Q, _ = np.linalg.qr(Km)
        c, *_ = np.linalg.lstsq(An @ Q, r0, rcond=None)
        expect = u0 + Q @ c
        got = orc.cgls(G, y.reshape(1, 10, 12), w.reshape(1, 10, 12), u0.reshape(1, 6, 6), m1=m).ravel()
        np.testing.assert_allclose(got, expect, rtol=1e-8, atol=1e-10)
        res = np.linalg.norm(yn - An @ got)
        assert res <= prev_res * (1 + 1e-12)
        prev_res = res
    # a run of 50 steps reaches the least-squares solution (36 unknowns, full
    # column rank, condition number ~6); far past convergence CGLS in floating
    # point loses conjugacy, so the run length stays moderate
    assert np.linalg.matrix_rank(An) == An.shape[1]
    ls, *_ = np.linalg.lstsq(An, yn, rcond=None)
    got = orc.cgls(G, y.reshape(1, 10, 12), w.reshape(1, 10, 12), u0.reshape(1, 6, 6), m1=50).ravel()
    np.testing.assert_allclose(got, ls, rtol=1e-6, atol=1e-8)


def test_P6_zero_residual_keeps_u(orc):
    geom = small_geom(N=2, L=8, V=12, B=16)
    G = orc.Geometry(geom)
    f = synth.configs.random_images((2, 8, 8), 6)
    y = orc.project(G, f)
    w = np.ones_like(y)
    assert np.array_equal(orc.cgls(G, y, w, f, m1=3), f)


def test_gradient_step_mode_eq4(orc):
    geom = small_geom(N=1, L=6, V=10, B=12)
    G = orc.Geometry(geom)
    A = dense_P_oracle(orc, geom)
    rng = np.random.default_rng(7)
    w = rng.uniform(0.5, 2.0, size=A.shape[0])
    y = rng.uniform(0, 3, size=A.shape[0])
    f = rng.uniform(0, 0.02, size=A.shape[1])
    beta = 1e4
    expect = f - (A.T @ (w * (A @ f - y))) / beta
    got = orc.cgls(G, y.reshape(1, 10, 12), w.reshape(1, 10, 12), f.reshape(1, 6, 6), m1=0, beta=beta)
    np.testing.assert_allclose(got.ravel(), expect, rtol=1e-12, atol=1e-14)


# -------------------------------------------------------------------- weights
def nlm_integral_image(gi, gj, d, W, h):
    """Weighted average sum_y w(x,y) gj(y) by per-offset box sums (cumulative sums)."""
    L = gi.shape[0]
    s, R = d // 2, W // 2
    idx = np.clip(np.arange(-s - R, L + s + R), 0, L - 1)
    Gi = gi[np.ix_(idx, idx)]
    Gj = gj[np.ix_(idx, idx)]
    off = s + R
    Ds, valid = [], []
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            # E(z) = (gi(clamp z) - gj(clamp(z + delta)))^2 on z in [-s, L+s)
            zi = np.arange(-s, L + s)
            a = Gi[np.ix_(zi + off, zi + off)]
            b = gj[np.ix_(np.clip(zi + dy, 0, L - 1), np.clip(zi + dx, 0, L - 1))]
            E = (a - b) ** 2
            cs = np.zeros((E.shape[0] + 1, E.shape[1] + 1))
            cs[1:, 1:] = E.cumsum(0).cumsum(1)
            Dm = cs[d:, d:] - cs[:-d, d:] - cs[d:, :-d] + cs[:-d, :-d]
            rr, cc = np.meshgrid(np.arange(L) + dy, np.arange(L) + dx, indexing="ij")
            valid.append((rr >= 0) & (rr < L) & (cc >= 0) & (cc < L))
            Ds.append(Dm)
    Ds = np.stack(Ds)
    valid = np.stack(valid)
    Ds = np.where(valid, Ds, np.inf)
    m = Ds.min(0)
    wts = np.where(valid, np.exp(-(Ds - m) / h ** 2), 0.0)
    wts /= wts.sum(0)
    out = np.zeros((L, L))
    k = 0
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            vj = gj[np.clip(np.arange(L) + dy, 0, L - 1)][:, np.clip(np.arange(L) + dx, 0, L - 1)]
            out += wts[k] * vj
            k += 1
    return out, wts, valid


def test_P7_weights_normalised_in_unit_interval(orc):
    g = synth.configs.smooth_random_images((2, 20, 20), 77)
    for (r, c) in [(0, 0), (3, 17), (10, 10), (19, 19)]:
        w, D = orc.weights(g[0], g[1], r, c, 5, 9, 0.004)
        ok = ~np.isnan(w)
        assert abs(w[ok].sum() - 1.0) < 1e-14
        assert (w[ok] > 0).all() and (w[ok] <= 1.0).all()
        # the number of candidates is the window truncated to the image
        assert ok.sum() == (min(r + 4, 19) - max(r - 4, 0) + 1) * (min(c + 4, 19) - max(c - 4, 0) + 1)


def test_P8_constant_is_fixed_point(orc):
    g = np.full((4, 16, 16), 0.017)
    out = orc.regularize(g, g, g, 5, 9, 0.003, 0.8)
    np.testing.assert_allclose(out, 0.017, rtol=1e-15, atol=0)


def test_P9_convex_combination_bounds(orc):
    rng = np.random.default_rng(9)
    g = rng.uniform(-0.01, 0.03, size=(3, 14, 14))
    d, W, R = 3, 7, 3
    out = orc.regularize(g, g, g, d, W, 0.01, 1.3, clamp=False)
    N, L = g.shape[0], g.shape[-1]
    for i in range(N):
        for r in range(L):
            for c in range(L):
                vals = [g[i, r, c]]
                for j in ((i - 1) % N, (i + 1) % N):
                    vals.append(g[j, max(r - R, 0):r + R + 1, max(c - R, 0):c + R + 1].ravel())
                vals = np.concatenate([np.atleast_1d(v) for v in vals])
                assert vals.min() - 1e-15 <= out[i, r, c] <= vals.max() + 1e-15


def test_P10_mu_zero_is_clamp(orc):
    rng = np.random.default_rng(10)
    g = rng.uniform(-0.01, 0.03, size=(3, 12, 12))
    out = orc.regularize(g, g, g, 5, 9, 0.01, 0.0, clamp=True)
    assert np.array_equal(out, np.maximum(g, 0.0))


def test_P11_infinite_h_is_window_mean(orc):
    rng = np.random.default_rng(11)
    g = rng.uniform(0, 0.03, size=(3, 12, 12))
    mu, R = 0.7, 3
    out = orc.regularize(g, g, g, 5, 2 * R + 1, 1e30, mu, clamp=False)
    N, L = 3, 12
    exp = np.empty_like(g)
    for i in range(N):
        for r in range(L):
            for c in range(L):
                a = sum(g[j, max(r - R, 0):r + R + 1, max(c - R, 0):c + R + 1].mean()
                        for j in ((i - 1) % N, (i + 1) % N))
                exp[i, r, c] = g[i, r, c] / (1 + mu) + mu / (2 * mu + 2) * a
    np.testing.assert_allclose(out, exp, rtol=1e-13, atol=1e-16)


def test_P12_motion_compensation_small_h(orc):
    rng = np.random.default_rng(12)
    L, d, W = 24, 3, 7
    base = rng.uniform(0, 0.03, size=(L + 10, L + 10))
    dl = (1, -2)   # shift between consecutive phases, |delta| <= window radius
    g = np.stack([base[5 - k * dl[0]:5 - k * dl[0] + L, 5 - k * dl[1]:5 - k * dl[1] + L] for k in range(3)])
    # g[k](x) = g[k-1](x - dl): phase 1 matches phase 0 at x - dl and phase 2 at x + dl
    out = orc.regularize(g, g, g, d, W, 1e-5, 0.9, clamp=False)
    m = 2 * 3 + 2
    np.testing.assert_allclose(out[1, m:-m, m:-m], g[1, m:-m, m:-m], rtol=1e-12, atol=1e-15)


def test_P13_single_phase_is_classical_nlm(orc):
    g = synth.configs.smooth_random_images((1, 18, 18), 13, passes=1)
    d, W, h, mu = 5, 9, 0.006, 1.1
    out = orc.regularize(g, g, g, d, W, h, mu, clamp=False)
    nl, _, _ = nlm_integral_image(g[0], g[0], d, W, h)
    expect = g[0] / (1 + mu) + mu / (2 * mu + 2) * 2 * nl
    np.testing.assert_allclose(out[0], expect, rtol=1e-11, atol=1e-15)


def patch_array(img, d):
    s = d // 2
    L = img.shape[0]
    idx = np.clip(np.arange(-s, L + s), 0, L - 1)
    P = img[np.ix_(idx, idx)]
    out = np.empty((L, L, d * d))
    k = 0
    for py in range(d):
        for px in range(d):
            out[:, :, k] = P[py:py + L, px:px + L]
            k += 1
    return out


def test_P14_dense_brute_force_8x8(orc):
    N, L, d, W, h, mu = 3, 8, 3, 5, 0.01, 0.6
    g = synth.configs.smooth_random_images((N, L, L), 14, passes=1)
    v = synth.configs.random_images((N, L, L), 140)
    out = orc.regularize(g, v, g, d, W, h, mu, clamp=False)
    R = W // 2
    P = [patch_array(g[i], d).reshape(L * L, -1) for i in range(N)]
    rr, cc = np.divmod(np.arange(L * L), L)
    win = (np.abs(rr[:, None] - rr[None]) <= R) & (np.abs(cc[:, None] - cc[None]) <= R)
    exp = np.empty((N, L * L))
    for i in range(N):
        acc = 0
        for j in ((i - 1) % N, (i + 1) % N):
            D = ((P[i][:, None, :] - P[j][None, :, :]) ** 2).sum(-1)      # 64 x 64
            D = np.where(win, D, np.inf)
            wts = np.exp(-(D - D.min(1, keepdims=True)) / h ** 2)
            wts /= wts.sum(1, keepdims=True)
            acc = acc + wts @ v[j].ravel()
        exp[i] = g[i].ravel() / (1 + mu) + mu / (2 * mu + 2) * acc
    np.testing.assert_allclose(out.reshape(N, -1), exp, rtol=1e-12, atol=1e-16)


def omega_matrix(orc, gi, gj, d, W, h):
    L = gi.shape[0]
    R = W // 2
    Om = np.zeros((L * L, L * L))
    for r in range(L):
        for c in range(L):
            w, _ = orc.weights(gi, gj, r, c, d, W, h)
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    if not np.isnan(w[dy + R, dx + R]):
                        Om[r * L + c, (r + dy) * L + (c + dx)] = w[dy + R, dx + R]
    return Om


def test_P15_gauss_jacobi_converges_to_linear_solve(orc):
    N, L, d, W, h, mu = 3, 8, 3, 5, 0.008, 1.5
    g = synth.configs.smooth_random_images((N, L, L), 15, passes=1) + 0.005
    n = L * L
    A = (1 + mu) * np.eye(N * n)
    for i in range(N):
        for j in ((i - 1) % N, (i + 1) % N):
            A[i * n:(i + 1) * n, j * n:(j + 1) * n] -= mu / 2 * omega_matrix(orc, g[i], g[j], d, W, h)
    ustar = np.linalg.solve(A, (g.ravel()))
    prev = np.abs(g.ravel() - ustar).max()
    ratio = mu / (1 + mu)
    for m in range(1, 8):
        um = orc.gauss_jacobi(g, d, W, h, mu, m2=m).ravel()
        err = np.abs(um - ustar).max()
        assert err <= ratio * prev * (1 + 1e-9) + 1e-15
        prev = err
    u = orc.gauss_jacobi(g, d, W, h, mu, m2=200).ravel()
    np.testing.assert_allclose(u, ustar, rtol=1e-12, atol=1e-15)


def test_P16_unnormalised_weights_symmetric(orc):
    g = synth.configs.smooth_random_images((2, 16, 16), 16)
    d, W, R = 5, 9, 4
    for (r, c) in [(2, 3), (8, 8), (15, 0)]:
        _, Dij = orc.weights(g[0], g[1], r, c, d, W, 0.01)
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                r2, c2 = r + dy, c + dx
                if 0 <= r2 < 16 and 0 <= c2 < 16:
                    _, Dji = orc.weights(g[1], g[0], r2, c2, d, W, 0.01)
                    assert Dij[dy + R, dx + R] == Dji[R - dy, R - dx]


def test_P17_equivariances(orc):
    g = synth.configs.smooth_random_images((5, 14, 14), 17, passes=1)
    v = synth.configs.random_images((5, 14, 14), 170)
    run = lambda a, b: orc.regularize(a, b, a, 3, 7, 0.006, 0.9, clamp=False)  # noqa: E731
    base = run(g, v)
    for tf in [lambda x: np.roll(x, 2, axis=0), lambda x: x[::-1], lambda x: x.transpose(0, 2, 1),
               lambda x: x[:, ::-1], lambda x: x[:, :, ::-1]]:
        np.testing.assert_allclose(run(tf(g).copy(), tf(v).copy()), tf(base), rtol=1e-12, atol=1e-16)


# ------------------------------------------------------------------------ FBP
def test_P18_fbp_scale_and_linearity(orc):
    geom = synth.ScanGeometry(n_phases=2, L=128, n_views=180, n_bins=512)
    mu0 = 0.02
    disk = [Ellipse(0.0, 0.0, 100.0, 100.0, 0.0, mu0)]
    src, u = geom.rays()
    y = ellipse_line_integrals(src, u, disk)
    G = orc.Geometry(geom)
    f = orc.fbp(G, y)
    assert np.array_equal(f[0], f[1])
    D = geom.pixel_mm
    k = (np.arange(128) + 0.5) * D - 250.0
    X, Y = np.meshgrid(k, k)
    inner = X ** 2 + Y ** 2 < (0.8 * 100.0) ** 2
    outer = X ** 2 + Y ** 2 > (1.2 * 100.0) ** 2
    assert abs(f[0][inner].mean() / mu0 - 1) < 0.02
    assert abs(f[0][outer].mean()) < 0.01 * mu0 and abs(f[0][outer]).mean() < 0.05 * mu0
    np.testing.assert_allclose(orc.fbp(G, 2 * y), 2 * f, rtol=1e-12, atol=1e-18)
    assert np.all(orc.fbp(G, np.zeros_like(y)) == 0)
    fp = orc.fbp(G, y, all_phases=False)   # each phase from its own 180 views
    assert abs(fp[1][inner].mean() / mu0 - 1) < 0.02


# ----------------------------------------------------------------------- cost
def test_P19_cost_invariants(orc):
    geom = small_geom(N=3, L=12, V=16, B=24)
    G = orc.Geometry(geom)
    f = synth.configs.smooth_random_images((3, 12, 12), 19)
    y = orc.project(G, f)
    w = np.ones_like(y)
    prm = orc.params(patch=3, window=5, h=0.01, mu_hat=1.0)
    data, reg = orc.cost(G, prm, y, w, f, f)
    assert data == 0.0 and reg > 0.0
    c = np.full_like(f, 0.013)
    data, reg = orc.cost(G, prm, orc.project(G, c), w, c, f)
    assert data == 0.0 and reg == 0.0


# ---------------------------------------------------------------- outer loop
def test_P20_resume_is_exact(orc):
    case = synth.make_case("C1", L=32, V=30, B=48, patch=3, window=7)
    G = orc.Geometry(case.geom)
    p4 = orc.case_params(case, max_outer=4)
    p2 = orc.case_params(case, max_outer=2)
    f4, k4, _, _ = orc.solve(G, p4, case.y, case.w)
    f2, _, _, _ = orc.solve(G, p2, case.y, case.w)
    f22, _, _, _ = orc.solve(G, p2, case.y, case.w, f0=f2)
    assert k4 == 4 and np.array_equal(f4, f22)


def test_solve_stops_at_tolerance(orc):
    case = synth.make_case("C1", L=32, V=30, B=48, patch=3, window=7)
    G = orc.Geometry(case.geom)
    f, k, rel, hist = orc.solve(G, orc.case_params(case, max_outer=30, tol=5e-3), case.y, case.w)
    assert rel < 5e-3 and k < 30 and (hist[:-1] >= 5e-3).all()


def test_cost_decreases_each_outer_iteration_C1(orc):
    """Empirical property (Eq. 6 omits the terms where f_i is J's second argument,
    so no monotone decrease is proven): checked for the C1 workload defaults."""
    case = synth.make_case("C1")
    G = orc.Geometry(case.geom)
    beta = orc.power_beta(G, case.w, 20)
    prm = orc.case_params(case, beta=beta)
    f = orc.fbp(G, case.y)
    costs = []
    for _ in range(6):
        g = orc.cgls(G, case.y, case.w, f, 3)
        f, _ = orc.step(G, prm, case.y, case.w, f)
        data, reg = orc.cost(G, prm, case.y, case.w, f, g)
        costs.append(data + case.mu_hat * beta / 2 * reg)
    assert all(b < a for a, b in zip(costs, costs[1:])), costs


def test_fixed_guide_of_constant_image_gives_window_means():
    """Weights taken from a fixed guide (Eq. 3 with a given image): for a
    constant guide every patch distance is 0, so each weight is 1 over the
    window truncated to the image, and one Gauss-Jacobi sweep of Eq. 7 is the
    plain window mean of the neighbour phases (computed here directly)."""
    import oracle
    N, L, d, W, mu = 4, 13, 3, 5, 0.7
    rng = np.random.default_rng(31)
    g = rng.uniform(0.0, 0.03, size=(N, L, L))
    guide = np.full((N, L, L), 0.0123)
    out = oracle.gauss_jacobi(g, d, W, 0.01, mu, m2=1, guide=guide)
    R = W // 2
    expect = np.empty_like(g)
    for i in range(N):
        for r in range(L):
            for c in range(L):
                rs, cs = slice(max(r - R, 0), min(r + R, L - 1) + 1), slice(max(c - R, 0), min(c + R, L - 1) + 1)
                m = g[(i - 1) % N][rs, cs].mean() + g[(i + 1) % N][rs, cs].mean()
                expect[i, r, c] = max(g[i, r, c] / (1 + mu) + mu / (2 * mu + 2) * m, 0.0)
    np.testing.assert_allclose(out, expect, rtol=1e-12, atol=1e-15)
    # and the weights from g itself differ (the guide is really used)
    assert np.abs(oracle.gauss_jacobi(g, d, W, 0.01, mu, m2=1) - expect).max() > 1e-6


# ------------------------------------------- composition of one outer iteration
def dense_weights(gi, gj, d, W, h):
    """Eq. 8 weights as an [L*L, L*L] matrix: plain SSD of edge-clamped d x d
    patches, the W x W window truncated to the image, softmax over it."""
    L = gi.shape[0]
    R = W // 2
    Pi = patch_array(gi, d).reshape(L * L, -1)
    Pj = patch_array(gj, d).reshape(L * L, -1)
    rr, cc = np.divmod(np.arange(L * L), L)
    win = (np.abs(rr[:, None] - rr[None]) <= R) & (np.abs(cc[:, None] - cc[None]) <= R)
    D = ((Pi[:, None, :] - Pj[None, :, :]) ** 2).sum(-1)
    D = np.where(win, D, np.inf)
    wts = np.exp(-(D - D.min(1, keepdims=True)) / h ** 2)
    return wts / wts.sum(1, keepdims=True)


def krylov_cgls(A, w, y, u0, m):
    """The m-th CGLS iterate as the minimiser of ||sqrt(w)(y - A u)|| over
    u0 + K_m(A_n^T A_n, A_n^T r0) (dense basis, no CGLS recurrences)."""
    An = np.sqrt(w)[:, None] * A
    r0 = np.sqrt(w) * y - An @ u0
    v = An.T @ r0
    K = []
    for _ in range(m):
        K.append(v / np.linalg.norm(v))
        v = An.T @ (An @ K[-1])
    Q, _ = np.linalg.qr(np.stack(K, 1))
    c, *_ = np.linalg.lstsq(An @ Q, r0, rcond=None)
    return u0 + Q @ c


def dense_outer_iteration(A, geom, y, w, f, m1, m2, d, W, h, mu):
    """One iteration of the TNLM algorithm box from dense matrices: g = CGLS
    (M1 steps, per phase); weights from g (Eq. 8); M2 Jacobi sweeps of Eq. 7
    from u = g with those weights; f = max(u, 0); and the relative update."""
    N, L, VB = geom.n_phases, geom.L, geom.n_views * geom.n_bins
    n = L * L
    g = np.stack([krylov_cgls(A[i * VB:(i + 1) * VB, i * n:(i + 1) * n], w[i].ravel(), y[i].ravel(),
                              f[i].ravel(), m1) for i in range(N)])
    Om = {(i, j): dense_weights(g[i].reshape(L, L), g[j].reshape(L, L), d, W, h)
          for i in range(N) for j in ((i - 1) % N, (i + 1) % N)}
    u = g.copy()
    for _ in range(m2):
        u = np.stack([g[i] / (1 + mu) + mu / (2 * mu + 2) * (Om[i, (i - 1) % N] @ u[(i - 1) % N] +
                                                             Om[i, (i + 1) % N] @ u[(i + 1) % N])
                      for i in range(N)])
    fn = np.maximum(u, 0.0).reshape(N, L, L)
    rel = np.linalg.norm(fn - f) / np.linalg.norm(fn)
    return fn, rel, g.reshape(N, L, L)


def _dense_problem(seed, N=3, L=6, V=10, B=12):
    geom = small_geom(N=N, L=L, V=V, B=B)
    A = dense_P_clip(geom)
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 2.0, size=(N, V, B))
    f0 = synth.configs.smooth_random_images((N, L, L), seed, passes=1)
    # data of an image with negative pixels, so the data step leaves negative
    # pixels and the place of the positivity clamp matters
    z = rng.normal(-0.01, 0.02, size=f0.shape)
    y = (A @ (f0 + z).ravel()).reshape(N, V, B) + rng.normal(0.0, 0.05, size=(N, V, B))
    return geom, A, y, w, f0


def test_step_is_cgls_then_jacobi_then_clamp(orc):
    """orc_step = CGLS from f^(k-1) (M1 = 3) -> weights from its output g ->
    M2 = 2 Jacobi sweeps starting at g -> clamp, and the relative update
    ||f^k - f^(k-1)|| / ||f^k|| (TNLM and Gauss-Jacobi boxes), against the
    dense composition above."""
    geom, A, y, w, f0 = _dense_problem(21)
    d, W, h, mu = 3, 5, 0.02, 0.8
    G = orc.Geometry(geom)
    prm = orc.params(patch=d, window=W, h=h, mu_hat=mu, m1=3, m2=2)
    got, rel = orc.step(G, prm, y, w, f0)
    exp, rel_exp, g = dense_outer_iteration(A, geom, y, w, f0, 3, 2, d, W, h, mu)
    assert g.min() < -0.01 and (exp == 0).sum() > 5     # the clamp acts after the sweeps
    np.testing.assert_allclose(got, exp, rtol=1e-9, atol=1e-12)
    assert abs(rel - rel_exp) <= 1e-9 * rel_exp
    # the alternatives that this composition excludes differ by far more
    # than the tolerance: weights or values from f^(k-1), clamp before the sweeps
    alt_guide = orc.gauss_jacobi(g, d, W, h, mu, m2=2, guide=f0)
    alt_clamp = orc.gauss_jacobi(np.maximum(g, 0), d, W, h, mu, m2=2)
    assert np.abs(alt_guide - exp).max() > 1e-4 and np.abs(alt_clamp - exp).max() > 1e-4


def test_solve_is_fbp_then_steps(orc):
    """orc_solve = f^(0) (FBP of all phases, or the caller's image) followed by
    outer iterations; the history holds each iteration's relative update."""
    geom, A, y, w, f0 = _dense_problem(22)
    d, W, h, mu = 3, 5, 0.02, 0.8
    G = orc.Geometry(geom)
    prm = orc.params(patch=d, window=W, h=h, mu_hat=mu, m1=2, m2=1, max_outer=3)
    f, k, rel, hist = orc.solve(G, prm, y, w, f0=f0)
    fe, rels = f0.copy(), []
    for _ in range(3):
        fe, r, _ = dense_outer_iteration(A, geom, y, w, fe, 2, 1, d, W, h, mu)
        rels.append(r)
    assert k == 3
    np.testing.assert_allclose(f, fe, rtol=1e-8, atol=1e-11)
    np.testing.assert_allclose(hist, rels, rtol=1e-8)
    assert rel == hist[-1]
    # from the FBP of all phases: the same iterations from that image
    f_fbp, k2, _, _ = orc.solve(G, prm, y, w)
    fe = orc.fbp(G, y)
    for _ in range(3):
        fe, _ = orc.step(G, prm, y, w, fe)
    assert k2 == 3 and np.array_equal(f_fbp, fe)


# ----------------------------------------------------------------------- cost
def test_cost_terms_against_dense_definition(orc):
    """Eq. 1 with Eq. 2: data = sum (P f - y)^T S^-1 (P f - y) with S^-1 =
    diag(w) (not its square root); reg = sum_i sum_{j = i+-1} sum_x sum_y
    w_ij(x, y) (f_i(x) - f_j(y))^2, the weights from the guide, not from f."""
    geom, A, y, w, f = _dense_problem(23)
    N, L = geom.n_phases, geom.L
    d, W, h = 3, 5, 0.015
    guide = synth.configs.smooth_random_images((N, L, L), 230, passes=1)
    G = orc.Geometry(geom)
    prm = orc.params(patch=d, window=W, h=h, mu_hat=1.0)
    data, reg = orc.cost(G, prm, y, w, f, guide)
    res = A @ f.ravel() - y.ravel()
    np.testing.assert_allclose(data, np.sum(w.ravel() * res * res), rtol=1e-12)
    exp = 0.0
    for i in range(N):
        for j in ((i - 1) % N, (i + 1) % N):
            Om = dense_weights(guide[i], guide[j], d, W, h)
            diff = f[i].ravel()[:, None] - f[j].ravel()[None, :]
            exp += np.sum(Om * diff * diff)
    np.testing.assert_allclose(reg, exp, rtol=1e-12)


# ---------------------------------------------------------------------- beta
def test_power_beta_is_largest_eigenvalue(orc):
    """beta of Eq. 4: the largest eigenvalue of P_i^T S^-1 P_i, maximised over
    phases (eigvalsh of the dense matrix). The power estimate never exceeds
    it and does not decrease with more iterations."""
    geom = small_geom(N=2, L=6, V=10, B=12)
    A = dense_P_clip(geom)
    rng = np.random.default_rng(24)
    w = rng.uniform(0.5, 2.0, size=(2, 10, 12))
    w[1] *= 3.0                                        # phase 1 holds the maximum
    VB, n = 120, 36
    lam = [np.linalg.eigvalsh(A[i * VB:(i + 1) * VB, i * n:(i + 1) * n].T @
                              (w[i].ravel()[:, None] * A[i * VB:(i + 1) * VB, i * n:(i + 1) * n]))[-1]
           for i in range(2)]
    G = orc.Geometry(geom)
    est = [orc.power_beta(G, w, k) for k in (2, 5, 30, 400)]
    assert all(e <= max(lam) * (1 + 1e-12) for e in est)
    assert all(b >= a * (1 - 1e-12) for a, b in zip(est, est[1:]))
    assert abs(est[-1] - max(lam)) <= 1e-9 * max(lam)
    assert lam[1] > lam[0]


# ------------------------------------------------------------------------ FBP
def test_fbp_detector_offset_sign(orc):
    """The FBP places the bins where the projector puts them: data taken with a
    quarter-bin detector offset and reconstructed with that offset come out
    sharper than when reconstructed with the opposite offset (a half-bin
    error in the back-projection smears every point over a ring)."""
    import dataclasses
    geom = synth.ScanGeometry(n_phases=1, L=128, n_views=360, n_bins=256, fov_mm=64.0)
    obj = [Ellipse(9.0, -6.0, 4.0, 4.0, 0.0, 0.02), Ellipse(-10.0, 8.0, 6.0, 3.0, 0.5, 0.015)]
    src, u = geom.rays()
    y = ellipse_line_integrals(src, u, obj)[None]
    truth = rasterize(obj, geom.L, geom.fov_mm, supersample=8)
    err = {}
    for off in (0.25, -0.25):
        g = dataclasses.replace(geom, det_offset_bins=off)
        f = orc.fbp(orc.Geometry(g), y)[0]
        err[off] = np.linalg.norm(f - truth) / np.linalg.norm(truth)
    assert err[0.25] < 0.8 * err[-0.25], err
    assert err[0.25] < 0.35, err   # edges of the ellipses limit the error of a band-limited FBP
