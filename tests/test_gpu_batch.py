"""Batched engine (many slices of uneven L, V, B in one launch per stage,
one outer iteration per replayed hipGraph) and the tile autotuner.

A batch must give, per slice, bitwise the result of the single-slice context
(same kernels, same per-slice arithmetic and reduction order), match the FP64
oracle within the trajectory bar, and let converged slices drop out while the
others go on.
"""
import os

import numpy as np
import pytest

import synth
from gpu_common import announce, f32, recon_for, rel_l2_per_phase, to_dev, to_host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


SHAPES = [dict(L=48, V=40, B=64, I0=1e4), dict(L=64, V=30, B=96, I0=3e4), dict(L=40, V=56, B=72, I0=5e5),
          dict(L=33, V=25, B=61, I0=2e4)]


def make_cases(K, tol=0.0):
    return [synth.make_case("C1", slice_index=s, K=K, tol=tol, patch=5, window=9, randomize=True, **sh)
            for s, sh in enumerate(SHAPES)]


def batch_for(cases, **kw):
    from paper_1009_1351_amd import Batch
    c = cases[0]
    return Batch([c.geom for c in cases], patch=c.patch, window=c.window, h=c.h, mu_hat=c.mu_hat,
                 max_outer=c.max_outer, tol=c.tol, **kw)


def test_batch_equals_single_slices_bitwise():
    cases = make_cases(K=4)
    bt = batch_for(cases)
    ys = [to_dev(c.y) for c in cases]
    ws = [to_dev(c.w) for c in cases]
    fs, iters, rel, sts, st = bt.solve(ys, ws)
    assert st == 0 and iters == [4] * len(cases)
    for c, y, w, f in zip(cases, ys, ws, fs):
        rc = recon_for(c.geom, patch=c.patch, window=c.window, h=c.h, mu_hat=c.mu_hat, max_outer=4)
        f1, k, _, _ = rc.solve(y, w)
        assert torch.equal(f, f1), c.name


def test_batch_matches_oracle(orc):
    cases = make_cases(K=3)
    bt = batch_for(cases)
    fs, iters, _, _, st = bt.solve([to_dev(c.y) for c in cases], [to_dev(c.w) for c in cases])
    for c, f in zip(cases[:2], fs[:2]):
        prm = orc.case_params(c, h=float(np.float32(c.h)), mu_hat=float(np.float32(c.mu_hat)))
        ref, _, _, _ = orc.solve(orc.Geometry(c.geom), prm, f32(c.y), f32(c.w))
        err = rel_l2_per_phase(to_host(f), ref)
        announce(f"batch vs oracle {c.name}: {err.max():.2e}")
        assert err.max() < 1e-4


def test_batch_slices_stop_independently():
    tol = 3e-3
    cases = make_cases(K=40, tol=tol)
    bt = batch_for(cases)
    fs, iters, rel, sts, st = bt.solve([to_dev(c.y) for c in cases], [to_dev(c.w) for c in cases])
    assert all(s == 0 for s in sts) and all(r < tol for r in rel)
    singles = []
    for c in cases:
        rc = recon_for(c.geom, patch=c.patch, window=c.window, h=c.h, mu_hat=c.mu_hat, max_outer=40, tol=tol)
        _, k, _, _ = rc.solve(to_dev(c.y), to_dev(c.w))
        singles.append(k)
    announce(f"iterations to tol: batch {iters}, single {singles}")
    assert iters == singles
    assert len(set(iters)) > 1, "the test wants slices that converge at different iterations"


def test_graph_replay_matches_direct_launches(monkeypatch):
    case = synth.make_case("C1", K=5)
    y, w = to_dev(case.y), to_dev(case.w)
    kw = dict(patch=case.patch, window=case.window, h=case.h, mu_hat=case.mu_hat, max_outer=5)
    a, _, _, _ = recon_for(case.geom, **kw).solve(y, w)
    monkeypatch.setenv("TNLM_NO_GRAPH", "1")
    b, _, _, _ = recon_for(case.geom, **kw).solve(y, w)
    assert torch.equal(a, b)
    # several solves replay the same graph; eager work and syncs in between
    rc = recon_for(case.geom, **kw)
    monkeypatch.delenv("TNLM_NO_GRAPH")
    rc2 = recon_for(case.geom, **kw)
    f = rc2.new_image()
    for _ in range(3):
        out, _, _, _ = rc2.solve(y, w, f)
        torch.cuda.synchronize()
        _ = (out * 2).sum().item()
        assert torch.equal(out, a)


def test_autotune_keeps_results_bitwise(tmp_path, monkeypatch):
    monkeypatch.setenv("TNLM_AUTOTUNE_CACHE", str(tmp_path / "tune.jsonl"))
    case = synth.make_case("C1", K=3)
    y, w = to_dev(case.y), to_dev(case.w)
    kw = dict(patch=case.patch, window=case.window, h=case.h, mu_hat=case.mu_hat, max_outer=3)
    ref, _, _, _ = recon_for(case.geom, **kw).solve(y, w)
    rc = recon_for(case.geom, **kw)
    rpl, ms = rc.autotune()
    announce(f"autotune: rows/lane {rpl}, ms {ms}")
    assert rpl in (4, 8) and all(m > 0 for m in ms)
    out, _, _, _ = rc.solve(y, w)
    assert torch.equal(out, ref)
    assert (tmp_path / "tune.jsonl").exists()
    # a new context of the same class starts from the cached choice and agrees
    out2, _, _, _ = recon_for(case.geom, **kw).solve(y, w)
    assert torch.equal(out2, ref)
    for rows in ("4", "8"):
        monkeypatch.setenv("TNLM_ROWS_PER_LANE", rows)
        o, _, _, _ = recon_for(case.geom, **kw).solve(y, w)
        assert torch.equal(o, ref), rows


def test_benchmark_batch_matches_single_slices_and_oracle(orc):
    """The benchmark's own launch configuration: dose cases a, b, c of the
    256^2 workload (360/60/60 views x 512 bins, patch 7, window 15) in one
    batch, with its cost-cut XCD ranges. Two outer iterations equal the
    single-slice contexts bitwise; the first iteration of dose case c matches
    the FP64 oracle (whole CGLS output, sampled regulariser outputs)."""
    from paper_1009_1351_amd import Batch
    announce("benchmark batch (C2 a/b/c)")
    cases = [synth.make_case(n, K=2) for n in ("C2a", "C2b", "C2c")]
    c0 = cases[0]
    kw = dict(patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat, max_outer=2)
    ys = [to_dev(c.y) for c in cases]
    ws = [to_dev(c.w) for c in cases]
    bt = Batch([c.geom for c in cases], **kw)
    fs, iters, _, sts, st = bt.solve(ys, ws)
    assert st == 0 and iters == [2, 2, 2]
    for c, y, w, f in zip(cases, ys, ws, fs):
        rc = recon_for(c.geom, **kw)
        f1, _, _, _ = rc.solve(y, w)
        assert torch.equal(f, f1), c.name
    # dose case c, one iteration, against the oracle
    c = cases[2]
    y, w = f32(c.y), f32(c.w)
    G = orc.Geometry(c.geom)
    b1 = Batch([c.geom], **{**kw, "max_outer": 1})
    f_gpu = to_host(b1.solve([to_dev(y)], [to_dev(w)])[0][0])
    rc = recon_for(c.geom, patch=c.patch, window=c.window, h=c.h, mu_hat=c.mu_hat)
    f0 = to_host(rc.fbp(to_dev(y)))
    g = orc.cgls(G, y, w, f0, 3)
    g_gpu = to_host(rc.data_step(to_dev(y), to_dev(w), to_dev(f0)))
    assert rel_l2_per_phase(g_gpu, g).max() < 1e-5
    # regulariser on sampled pixels, from the GPU's own CGLS output (as in the kernel)
    rng = np.random.default_rng(11)
    h32, mu32 = float(np.float32(c.h)), float(np.float32(c.mu_hat))
    d, W, N, L = c.patch, c.window, 10, 256
    R = W // 2
    for _ in range(16):
        i, r, col = int(rng.integers(N)), int(rng.integers(L)), int(rng.integers(L))
        acc = 0.0
        for j in ((i - 1) % N, (i + 1) % N):
            wts, _ = orc.weights(g_gpu[i], g_gpu[j], r, col, d, W, h32)
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    if not np.isnan(wts[dy + R, dx + R]):
                        acc += wts[dy + R, dx + R] * g_gpu[j, r + dy, col + dx]
        expect = max(g_gpu[i, r, col] / (1 + mu32) + mu32 / (2 * mu32 + 2) * acc, 0.0)
        assert abs(f_gpu[i, r, col] - expect) <= 1e-5 * max(abs(expect), 1e-3), (i, r, col)


def test_batched_workload_shapes_equal_single_slices():
    """Slices of the batched workload at their real shapes (L 128 / 384 / 256 /
    512, 48-230 views, B = 1.5 L), mixed in one batch: each equals its
    single-slice solve bitwise after two outer iterations."""
    from paper_1009_1351_amd import Batch
    announce("batched workload shapes")
    idx = [6, 4, 8, 3]   # 128 x 48 views, 384 x 61, 256 x 109, 512 x 230
    cases = [synth.make_case("C3", slice_index=s, K=2) for s in idx]
    c0 = cases[0]
    kw = dict(patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat, max_outer=2)
    ys = [to_dev(c.y) for c in cases]
    ws = [to_dev(c.w) for c in cases]
    fs, iters, _, _, st = Batch([c.geom for c in cases], **kw).solve(ys, ws)
    assert st == 0 and iters == [2] * len(cases)
    for c, y, w, f in zip(cases, ys, ws, fs):
        f1, _, _, _ = recon_for(c.geom, **kw).solve(y, w)
        assert torch.equal(f, f1), c.name


@pytest.mark.parametrize("N,L,d,W,same", [(4, 29, 3, 5, False), (3, 40, 3, 5, True), (3, 40, 5, 11, True),
                                          (2, 50, 9, 21, True), (5, 70, 7, 15, True)])
def test_tile_heights_agree_bitwise(monkeypatch, N, L, d, W, same):
    """Each pixel's arithmetic does not depend on the regulariser's tile height
    (4 or 8 output rows per lane), so the autotuner may pick either."""
    announce(f"tile heights N={N} L={L} d={d} W={W}")
    g = synth.configs.smooth_random_images((N, L, L), 200 + L, passes=1)
    v = g if same else synth.configs.random_images((N, L, L), 300 + L)
    gd, vd = to_dev(g), to_dev(v)
    outs = []
    for rows in ("8", "4"):
        monkeypatch.setenv("TNLM_ROWS_PER_LANE", rows)
        rc = recon_for(synth.ScanGeometry(n_phases=N, L=L, n_views=8, n_bins=16), patch=d, window=W, h=0.004,
                       mu_hat=0.7)
        outs.append(rc.regularize(gd, gd if same else vd, gd, clamp=False))
    assert torch.equal(outs[0], outs[1])


def test_active_mask_solves_a_subset():
    """tnlm_batch_solve_active: the active slices get exactly what a solve of
    the whole batch gives them, the others are left untouched."""
    cases = [synth.make_case("C1", slice_index=k, K=4) for k in range(3)]
    c0 = cases[0]
    kw = dict(patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat)
    ys = [to_dev(c.y) for c in cases]
    ws = [to_dev(c.w) for c in cases]
    f0 = [recon_for(c.geom, **kw).fbp(y) for c, y in zip(cases, ys)]
    from paper_1009_1351_amd import Batch
    bt = Batch([c.geom for c in cases], init="user", max_outer=4, tol=0.0, **kw)
    full, it_full, _, _, _ = bt.solve(ys, ws, [f.clone() for f in f0])
    part, it_part, _, st_part, _ = bt.solve(ys, ws, [f.clone() for f in f0], active=[True, False, True])
    assert torch.equal(part[0], full[0]) and torch.equal(part[2], full[2])
    assert torch.equal(part[1], f0[1])
    assert it_part == [4, 0, 4] and it_full == [4, 4, 4] and st_part[1] == 0
    # resuming the middle slice alone continues from its image
    rest, it_rest, _, _, _ = bt.solve(ys, ws, part, active=[False, True, False])
    assert it_rest == [0, 4, 0] and torch.equal(rest[1], full[1])

