"""Patch distances on the BF16 matrix cores (ssd_mode = "bf16_mfma").

The cross term of ||a||^2 + ||b||^2 - 2<a, b> comes from BF16 MFMAs with FP32
accumulation (centred values, hi/lo split, three products); exponentials and
the Gauss-Jacobi update stay FP32. The error against the FP64 oracle is
measured and printed per phase; the asserted bars are loose (the mode's error
is a reported quantity, not a parity claim).
"""
import numpy as np
import pytest

import synth
from gpu_common import announce, case_inputs, f32, recon_for, rel_l2_per_phase, to_dev, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def small_geom(N, L):
    return synth.ScanGeometry(n_phases=N, L=L, n_views=8, n_bins=16)


@pytest.mark.parametrize("N,L,d,W,h", [(3, 40, 5, 11, 0.004), (4, 37, 7, 15, 0.006), (3, 33, 3, 7, 0.003)])
def test_bf16_regularize_error(orc, N, L, d, W, h):
    g = f32(synth.configs.smooth_random_images((N, L, L), 500 + L, passes=1) + 0.01)
    rc = recon_for(small_geom(N, L), patch=d, window=W, h=h, mu_hat=0.7, ssd_mode="bf16_mfma")
    gd = to_dev(g)
    out = to_host(rc.regularize(gd, gd, gd, clamp=False))
    ref = orc.regularize(g, g, g, d, W, float(np.float32(h)), float(np.float32(0.7)), clamp=False)
    err = rel_l2_per_phase(out, ref)
    mx = np.abs(out - ref).max(axis=(1, 2)) / np.abs(ref).max()
    announce(f"bf16 regularize d={d} W={W}: rel L2 per phase {np.array2string(err, precision=2)}, "
             f"max abs / max {np.array2string(mx, precision=2)}")
    assert err.max() < 1e-3


def test_bf16_trajectory_error_C1(orc):
    case = synth.make_case("C1")
    y, w = case_inputs(case)
    prm = orc.case_params(case, h=float(np.float32(case.h)), mu_hat=float(np.float32(case.mu_hat)))
    ref, _, _, _ = orc.solve(orc.Geometry(case.geom), prm, y, w)
    rc = recon_for(case.geom, patch=case.patch, window=case.window, h=case.h, mu_hat=case.mu_hat,
                   max_outer=case.max_outer, ssd_mode="bf16_mfma")
    f, k, _, _ = rc.solve(to_dev(y), to_dev(w))
    err = rel_l2_per_phase(to_host(f), ref)
    announce(f"bf16 C1 trajectory: rel L2 per phase {np.array2string(err, precision=2)}")
    assert k == case.max_outer and err.max() < 5e-3


def test_bf16_precision_workload_sampled(orc):
    """Precision workload shape (10 phases, 512^2, 720 bins, 120 views, I0
    5e4, patch 7, window 15): one regulariser sweep with BF16-MFMA distances
    from the CGLS output of the FBP start, against the FP64 oracle's Eq. 7
    on sampled pixels; per-phase relative L2 and max error are printed."""
    case = synth.make_case("C4", slice_index=0)
    y, w = case_inputs(case)
    kw = dict(patch=case.patch, window=case.window, h=case.h, mu_hat=case.mu_hat)
    rc32 = recon_for(case.geom, **kw)
    rc16 = recon_for(case.geom, ssd_mode="bf16_mfma", **kw)
    yd, wd = to_dev(y), to_dev(w)
    gd = rc32.data_step(yd, wd, rc32.fbp(yd))
    g = to_host(gd)
    out16 = to_host(rc16.regularize(gd, gd, gd))
    out32 = to_host(rc32.regularize(gd, gd, gd))
    rng = np.random.default_rng(21)
    h32, mu32 = float(np.float32(case.h)), float(np.float32(case.mu_hat))
    d, W, N, L = case.patch, case.window, 10, case.geom.L
    R = W // 2
    exp_, got16, got32, ph = [], [], [], []
    for i in range(N):
        for _ in range(12):
            r, c = int(rng.integers(L)), int(rng.integers(L))
            acc = 0.0
            for j in ((i - 1) % N, (i + 1) % N):
                wts, _ = orc.weights(g[i], g[j], r, c, d, W, h32)
                for dy in range(-R, R + 1):
                    for dx in range(-R, R + 1):
                        if not np.isnan(wts[dy + R, dx + R]):
                            acc += wts[dy + R, dx + R] * g[j, r + dy, c + dx]
            exp_.append(max(g[i, r, c] / (1 + mu32) + mu32 / (2 * mu32 + 2) * acc, 0.0))
            got16.append(out16[i, r, c])
            got32.append(out32[i, r, c])
            ph.append(i)
    exp_, got16, got32, ph = map(np.asarray, (exp_, got16, got32, ph))
    rel16 = [np.linalg.norm(got16[ph == i] - exp_[ph == i]) / np.linalg.norm(exp_[ph == i]) for i in range(N)]
    mx16 = [np.abs(got16[ph == i] - exp_[ph == i]).max() / np.abs(exp_).max() for i in range(N)]
    rel32 = [np.linalg.norm(got32[ph == i] - exp_[ph == i]) / np.linalg.norm(exp_[ph == i]) for i in range(N)]
    announce("bf16 precision workload, sampled rel L2 per phase: " + " ".join(f"{e:.1e}" for e in rel16))
    announce("bf16 precision workload, sampled max abs / max per phase: " + " ".join(f"{e:.1e}" for e in mx16))
    announce("fp32 on the same samples, rel L2 per phase: " + " ".join(f"{e:.1e}" for e in rel32))
    assert max(rel32) < 1e-5
    assert max(rel16) < 1e-3
