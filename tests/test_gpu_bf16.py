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
