"""Coarse-to-fine start: the upsampling kernel against a reference
interpolation, and a two-level solve that reaches the tolerance at the
solution of the cold start (its iteration counts are printed: at 64^2 the
coarse start is not faster; the 512^2 comparison is a leg of the benchmark)."""
import numpy as np
import pytest

import synth
from gpu_common import announce, recon_for, to_dev

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
