"""The symmetric-reuse regulariser (ssd_mode "fp32_sym", §2.3) against the
FP64 oracle and against the per-phase FP32 kernel.

The oracle computes each direction of each phase pair on its own, with the
window-minimum shift of Eq. 8; the symmetric kernel computes each unordered
pair's distances and unshifted exponentials once for both directions, so the
two agree up to FP32 rounding (bar 1e-5 relative L2 per phase, as for the
FP32 kernel). Where the unshifted weights of a pixel underflow, the kernel
recomputes that pixel's direction exactly: a tiny h forces that path.
"""
import numpy as np
import pytest

import synth
from gpu_common import announce, f32, recon_for, rel_l2_per_phase, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SYM_CASES = [
    # N, L, d, W, h, mu, same guide/value
    (3, 40, 5, 11, 0.004, 0.5, True),
    (3, 37, 7, 15, 0.006, 1.0, True),
    (4, 29, 3, 5, 0.003, 0.7, False),
    (2, 50, 9, 19, 0.008, 2.0, True),
    (3, 45, 9, 19, 0.008, 1.5, False),
    (1, 35, 7, 9, 0.005, 0.9, False),
    (5, 70, 7, 15, 0.005, 0.5, True),
    (10, 100, 7, 15, 0.007, 0.5, False),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1009_1351_amd._native  # noqa: F401  (fails loudly when the library is missing)


def small_geom(N, L):
    return synth.ScanGeometry(n_phases=N, L=L, n_views=8, n_bins=16)


@pytest.mark.parametrize("N,L,d,W,h,mu,same", SYM_CASES)
def test_sym_regularize_matches_oracle(orc, N, L, d, W, h, mu, same):
    announce(f"sym regularize N={N} L={L} d={d} W={W} same={same}")
    g = f32(synth.configs.smooth_random_images((N, L, L), 200 + L, passes=1))
    v = g if same else f32(synth.configs.random_images((N, L, L), 300 + L))
    rc = recon_for(small_geom(N, L), patch=d, window=W, h=h, mu_hat=mu, ssd_mode="fp32_sym")
    gd = to_dev(g)
    out = to_host(rc.regularize(gd, gd if same else to_dev(v), gd, clamp=False))
    ref = orc.regularize(g, v, g, d, W, float(np.float32(h)), float(np.float32(mu)), clamp=False)
    err = rel_l2_per_phase(out, ref)
    announce(f"  rel L2 per phase max {err.max():.2e}")
    assert err.max() < 1e-5, err


def test_sym_matches_fp32_kernel():
    """Same inputs through both kernels: the results differ by rounding only."""
    N, L = 10, 130
    g = f32(synth.configs.smooth_random_images((N, L, L), 77, passes=2))
    gd = to_dev(g)
    outs = []
    for mode in ("fp32", "fp32_sym"):
        rc = recon_for(small_geom(N, L), patch=7, window=15, h=0.007, mu_hat=0.5, ssd_mode=mode)
        outs.append(to_host(rc.regularize(gd, gd, gd)))
    err = rel_l2_per_phase(outs[1], outs[0].astype(np.float64))
    announce(f"sym vs fp32 kernel: rel L2 per phase max {err.max():.2e}")
    assert err.max() < 2e-6


@pytest.mark.parametrize("h", [1e-4, 2.5e-3])
def test_sym_underflow_fallback(orc, h):
    """h = 1e-4: every pixel's best match lies thousands of h^2 away, all
    unshifted weights underflow and every pixel takes the exact path. h =
    2.5e-3 on an image that is flat on its left half and noisy on its right:
    only the noisy pixels take it, the flat ones keep the shared weights."""
    N, L = 3, 48
    rng = np.random.Generator(np.random.PCG64(99))
    g = 0.02 + 0.004 * rng.standard_normal((N, L, L))
    if h > 1e-3:
        g[:, :, : L // 2] = 0.02
    g = f32(g)
    rc = recon_for(small_geom(N, L), patch=5, window=9, h=h, mu_hat=0.8, ssd_mode="fp32_sym")
    gd = to_dev(g)
    out = to_host(rc.regularize(gd, gd, gd, clamp=False))
    ref = orc.regularize(g, g, g, 5, 9, float(np.float32(h)), float(np.float32(0.8)), clamp=False)
    err = rel_l2_per_phase(out, ref)
    announce(f"sym fallback h={h}: rel L2 per phase max {err.max():.2e}")
    assert np.isfinite(out).all()
    assert err.max() < 1e-5, err


def test_sym_batch_equals_single_slices():
    """A ragged batch (four sizes) gives each slice the bits the same slice
    gets alone: the work split and the fixed summation orders do not depend
    on the batch."""
    from paper_1009_1351_amd import Batch
    shapes = [dict(L=48, V=40, B=64, I0=1e4), dict(L=64, V=30, B=96, I0=3e4), dict(L=40, V=56, B=72, I0=5e5),
              dict(L=33, V=25, B=61, I0=2e4)]
    cases = [synth.make_case("C1", slice_index=s, K=3, tol=0.0, patch=5, window=9, randomize=True, **sh)
             for s, sh in enumerate(shapes)]
    c = cases[0]
    kw = dict(patch=c.patch, window=c.window, h=c.h, mu_hat=c.mu_hat, max_outer=3, ssd_mode="fp32_sym")
    bt = Batch([c.geom for c in cases], tol=0.0, **kw)
    ys = [to_dev(c.y) for c in cases]
    ws = [to_dev(c.w) for c in cases]
    fs, iters, _, _, st = bt.solve(ys, ws)
    assert st == 0 and iters == [3] * len(cases)
    for c, y, w, f in zip(cases, ys, ws, fs):
        rc = recon_for(c.geom, **kw)
        f1, _, _, _ = rc.solve(y, w)
        assert torch.equal(f, f1), c.name


def test_sym_trajectory_matches_oracle(orc):
    """Ten outer iterations of the 64^2 workload (FBP of all phases, CGLS,
    symmetric regulariser) against the oracle's solve: the trajectory bar."""
    case = synth.make_case("C1")
    y, w = f32(case.y), f32(case.w)
    rc = recon_for(case.geom, patch=case.patch, window=case.window, h=case.h, mu_hat=case.mu_hat,
                   max_outer=case.max_outer, ssd_mode="fp32_sym")
    f, k, _, _ = rc.solve(to_dev(y), to_dev(w))
    prm = orc.case_params(case, h=float(np.float32(case.h)), mu_hat=float(np.float32(case.mu_hat)))
    ref, kr, _, _ = orc.solve(orc.Geometry(case.geom), prm, y, w)
    err = rel_l2_per_phase(to_host(f), ref)
    announce(f"sym C1 trajectory vs oracle: {err.max():.2e}")
    assert k == kr and err.max() < 1e-4
