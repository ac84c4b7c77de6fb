"""Coarse-to-fine start: the upsampling kernel against a reference
interpolation, and a two-level solve that reaches the tolerance at the
solution of the cold start (its iteration counts are printed: at 64^2 the
coarse start is not faster; the 512^2 comparison is a leg of the benchmark)."""
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


@pytest.mark.parametrize("n,h,w,f", [(3, 17, 23, 2), (1, 32, 32, 4), (2, 5, 7, 3)])
def test_upsample_matches_bilinear_reference(n, h, w, f):
    import torch.nn.functional as F
    from paper_1009_1351_amd.multigrid import upsample
    x = to_dev(np.random.default_rng(n * h + w).uniform(0, 1, size=(n, h, w)))
    got = upsample(x, f)
    ref = F.interpolate(x[None].double(), scale_factor=f, mode="bilinear", align_corners=False)[0].float()
    assert got.shape == (n, h * f, w * f)
    assert float((got - ref).abs().max()) < 2e-6


def test_two_level_solve_reaches_the_cold_solution():
    from paper_1009_1351_amd.multigrid import MultigridSolver
    # the 64^2 workload converges steadily (its relative-update history is pinned
    # against the oracle); many larger slices settle into a period-2 cycle instead
    cases = [synth.make_case("C1")]
    c0 = cases[0]
    prm = dict(patch=c0.patch, window=c0.window, h=c0.h, mu_hat=c0.mu_hat)
    ys = [to_dev(c.y) for c in cases]
    ws = [to_dev(c.w) for c in cases]
    mg = MultigridSolver([c.geom for c in cases], tol=1e-4, max_outer=400, **prm)
    fm, it_f, it_c, st = mg.solve(ys, ws)
    for c, y, w, f, k, kc, s in zip(cases, ys, ws, fm, it_f, it_c, st):
        rc = recon_for(c.geom, max_outer=400, tol=1e-4, **prm)
        fcold, kcold, _, scold = rc.solve(y, w)
        d = float(torch.linalg.vector_norm(f - fcold) / torch.linalg.vector_norm(fcold))
        announce(f"{c.name}: cold {kcold} its; two-level {kc} coarse + {k} fine; difference {d:.2e}")
        assert s == 0 and scold == 0
        assert d < 2e-2   # both stop at relative update 1e-4, on different paths


def test_two_level_solve_matches_oracle_solve():
    """The oracle checks the coarse-to-fine path: its own cold solve of the
    64^2 workload to the same relative-update tolerance (stored by
    tests/golden/make_golden.py as c1tol). Both stop where the
    update falls below tol; with the contraction rho of the outer iteration
    measured from the oracle's last updates, each stopped iterate lies within
    about tol * rho / (1 - rho) of the fixed point, so the two agree to twice
    that (bar: three times, and at least 2e-3)."""
    from paper_1009_1351_amd.multigrid import MultigridSolver
    tol = 1e-4
    c = synth.make_case("C1")
    y, w = case_inputs(c)
    prm = dict(patch=c.patch, window=c.window, h=c.h, mu_hat=c.mu_hat)
    mg = MultigridSolver([c.geom], tol=tol, max_outer=400, **prm)
    fm, it_f, it_c, st = mg.solve([to_dev(y)], [to_dev(w)])
    mg.close()
    gold = _golden().load("c1tol")
    ref, hist = gold["f"].astype(np.float64), gold["hist"]
    kr, relr = int(gold["iters"]), float(hist[-1])
    rho = float(np.median(hist[-5:] / hist[-6:-1]))
    bar = max(2e-3, 3.0 * 2.0 * tol * rho / (1.0 - rho))
    d = rel_l2_per_phase(to_host(fm[0]), ref).max()
    announce(f"two-level {it_c[0]} coarse + {it_f[0]} fine vs oracle cold {kr} iterations; contraction {rho:.3f}; "
              f"max rel L2 per phase {d:.2e} (bar {bar:.2e})")
    assert st[0] == 0 and relr < tol and d < bar


def _golden():
    import importlib.util
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(here, "golden", "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    if not os.path.exists(mod.path("c1tol")):
        pytest.skip("stored result c1tol not generated")
    return mod
