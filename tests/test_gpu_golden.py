"""Full-size parity: the HIP path against stored FP64-oracle results.

The stored results (tests/golden/*.npz) are written by
tests/golden/make_golden.py, which calls only the oracle on the seeded
inputs; here the same inputs go through the C ABI, in the launch
configurations the benchmark uses (one slice per context; the 256^2 dose
cases as one batch; the 64-slice mixed batch), and every element is compared.

Bars (relative L2 per phase; the largest absolute error is reported):
  regulariser sweep, 10 x 256^2, patch 7, window 15 ....... 1e-5
  50-iteration trajectories (FP32) ......................... 1e-4  (the acceptance bar)
  50-iteration trajectory with BF16-MFMA patch distances ... reported; bar 1e-2
"""
import importlib.util
import os

import numpy as np
import pytest

import synth
from gpu_common import announce, case_inputs, f32, recon_for, rel_l2_per_phase, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
golden = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(golden)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1009_1351_amd._native  # noqa: F401  (fails loudly when the library is missing)


def stored(name):
    if not os.path.exists(golden.path(name)):
        pytest.skip(f"stored result {name} not generated")
    return golden.load(name)


def report(tag, got, ref):
    err = rel_l2_per_phase(got, ref)
    mx = np.abs(np.asarray(got, np.float64) - ref).max(axis=(1, 2))
    announce(f"{tag}: rel L2 per phase max {err.max():.2e} (mean {err.mean():.2e}); max abs per phase "
             f"max {mx.max():.2e} (image max {np.abs(ref).max():.3e})")
    return err, mx


@pytest.mark.parametrize("ssd_mode", ["fp32", "fp32_sym"])
def test_regulariser_sweep_256(ssd_mode):
    """One full-image regulariser sweep at the benchmark's shape: each of the
    persistent blocks handles several tiles here, so the tile loop and its LDS
    reuse are compared element by element (per-phase kernel, and the
    symmetric reuse of the phase pairs)."""
    ref = stored("sweep256")["f"].astype(np.float64)
    case, g = golden.sweep_input()
    rc = recon_for(case.geom, patch=case.patch, window=case.window, h=case.h, mu_hat=case.mu_hat,
                   ssd_mode=ssd_mode)
    gd = to_dev(g)
    out = to_host(rc.regularize(gd, gd, gd))
    err, _ = report(f"sweep 10 x 256^2 ({ssd_mode})", out, ref)
    assert err.max() < 1e-5


def _solve_single(name, ssd_mode="fp32"):
    gold = stored(name)
    config, s = golden.TRAJECTORIES[name]
    case = synth.make_case(config, slice_index=s)
    y, w = case_inputs(case)
    rc = recon_for(case.geom, patch=case.patch, window=case.window, h=case.h, mu_hat=case.mu_hat,
                   max_outer=case.max_outer, ssd_mode=ssd_mode)
    f, k, rel, status = rc.solve(to_dev(y), to_dev(w))
    return gold, case, to_host(f), k, rc.history()


@pytest.mark.parametrize("name", ["c2a", "c2b", "c2c"])
def test_trajectory_256_matches_oracle(name):
    """50 outer iterations of the paper-size slice from the FBP of all phases,
    one context per slice."""
    announce(f"trajectory {name}")
    gold, case, f, k, hist = _solve_single(name)
    err, _ = report(f"{name} 50 iterations", f, gold["f"].astype(np.float64))
    assert k == int(gold["iters"]) == case.max_outer
    assert err.max() < 1e-4
    np.testing.assert_allclose(hist, gold["hist"], rtol=2e-3)


def test_trajectory_256_symmetric_matches_oracle():
    """The low-dose 256^2 slice, 50 iterations, with the symmetric-reuse
    regulariser: the same stored oracle result and the same bar."""
    announce("trajectory c2c, symmetric reuse")
    gold, case, f, k, hist = _solve_single("c2c", ssd_mode="fp32_sym")
    err, _ = report("c2c 50 iterations (fp32_sym)", f, gold["f"].astype(np.float64))
    assert k == int(gold["iters"]) == case.max_outer
    assert err.max() < 1e-4
    np.testing.assert_allclose(hist, gold["hist"], rtol=2e-3)


def test_dose_cases_as_one_batch_match_oracle():
    """The three 256^2 dose cases solved together by the batched engine."""
    from paper_1009_1351_amd import Batch
    names = ["c2a", "c2b", "c2c"]
    golds = [stored(n) for n in names]
    cases = [synth.make_case(golden.TRAJECTORIES[n][0]) for n in names]
    c0 = cases[0]
    bt = Batch([c.geom for c in cases], patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat,
               max_outer=c0.max_outer)
    ys = [to_dev(f32(c.y)) for c in cases]
    ws = [to_dev(f32(c.w)) for c in cases]
    fs, iters, _, sts, _ = bt.solve(ys, ws)
    bt.close()
    for n, g, f, k in zip(names, golds, fs, iters):
        err, _ = report(f"batched {n}", to_host(f), g["f"].astype(np.float64))
        assert k == c0.max_outer and err.max() < 1e-4


_MIXED = []


def _mixed_batch_cases():
    if not _MIXED:
        _MIXED.extend(synth.make_case("C3", slice_index=s) for s in range(64))
    return _MIXED


@pytest.mark.parametrize("ssd_mode", ["fp32", "fp32_sym"])
def test_mixed_batch_slices_match_oracle(ssd_mode):
    """The 64-slice mixed batch of the benchmark (L from 128 to 512, 40-360
    views, 1.5 L bins), 50 iterations in one batched solve; the slices the
    oracle ran, one of each image size (128^2 with 48 views, 256^2 with 56,
    384^2 with 61, 512^2 with 48), are compared whole, and every slice's image
    must be finite and non-negative."""
    from paper_1009_1351_amd import Batch
    picks = {s: stored(f"c3s{s}") for s in (4, 6, 16, 34)}
    announce(f"mixed batch: 64 slices, 50 iterations ({ssd_mode})")
    cases = _mixed_batch_cases()
    c0 = cases[0]
    bt = Batch([c.geom for c in cases], patch=7, window=15, h=c0.h, mu_hat=c0.mu_hat, max_outer=50,
               ssd_mode=ssd_mode)
    ys = [to_dev(f32(c.y)) for c in cases]
    ws = [to_dev(f32(c.w)) for c in cases]
    fs, iters, _, sts, st = bt.solve(ys, ws)
    bt.close()
    assert st == 0 and all(k == 50 for k in iters)
    for s, g in picks.items():
        err, _ = report(f"mixed batch slice {s} (L {cases[s].geom.L}, {ssd_mode})", to_host(fs[s]),
                        g["f"].astype(np.float64))
        assert err.max() < 1e-4
    for f in fs:
        assert bool(torch.isfinite(f).all()) and float(f.min()) >= 0.0


def test_trajectory_512_matches_oracle():
    """Slice 0 of the 512^2 precision workload (120 views x 720 bins), 50
    iterations, FP32 patch distances."""
    announce("trajectory c4s0 fp32")
    gold, case, f, k, hist = _solve_single("c4s0")
    err, _ = report("c4s0 fp32 50 iterations", f, gold["f"].astype(np.float64))
    assert k == 50 and err.max() < 1e-4


def test_bf16_trajectory_512_error_reported():
    """The same slice with BF16-MFMA patch distances (FP32 accumulation,
    compensated split; exponentials and Gauss-Jacobi in FP32): per-phase
    error against the FP64 oracle over the 50-iteration trajectory."""
    announce("trajectory c4s0 bf16")
    gold, case, f, k, hist = _solve_single("c4s0", ssd_mode="bf16_mfma")
    err, mx = report("c4s0 bf16-mfma 50 iterations", f, gold["f"].astype(np.float64))
    announce("per phase rel L2: " + " ".join(f"{e:.2e}" for e in err))
    announce("per phase max abs: " + " ".join(f"{e:.2e}" for e in mx))
    assert k == 50 and err.max() < 1e-2
