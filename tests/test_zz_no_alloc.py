"""tnlm_regularize_noalloc (no context, no allocation; tables in a
library-owned device array) against the context entry point
tnlm_regularize on the same inputs: the same kernel and tiles, so the
outputs must be bitwise equal. Three calls in a row share the one array:
a 10 x 96^2 stack with a separate value stack, the same stack as guide =
value = g, then a smaller 3 x 40^2 stack with another patch and window."""
import ctypes as C

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
    import paper_1009_1351_amd._native  # noqa: F401  (fails loudly when the library is missing)


def _noalloc(N, L, patch, window, h, mu, guide, value, g, out, clamp=1):
    from paper_1009_1351_amd import _native as nat
    stream = torch.cuda.current_stream().cuda_stream
    st = nat.lib.tnlm_regularize_noalloc(N, L, patch, window, h, mu, C.c_void_p(guide.data_ptr()),
                                         C.c_void_p(value.data_ptr()), C.c_void_p(g.data_ptr()),
                                         C.c_void_p(out.data_ptr()), clamp, C.c_void_p(stream))
    nat.check(st)


def test_noalloc_regulariser_equals_context_entry_point():
    cases = [(10, 96, 7, 15, False, 11), (10, 96, 7, 15, True, 11), (3, 40, 5, 9, True, 21)]
    h, mu = 0.004, 0.5
    for N, L, patch, window, same, seed in cases:
        announce(f"noalloc regulariser N={N} L={L} patch={patch} window={window} same={same}")
        geom = synth.ScanGeometry(n_phases=N, L=L, n_views=8, n_bins=16)
        rc = recon_for(geom, patch=patch, window=window, h=h, mu_hat=mu)
        guide = to_dev(synth.configs.smooth_random_images((N, L, L), seed))
        value = guide if same else to_dev(synth.configs.smooth_random_images((N, L, L), seed + 1))
        g = guide if same else to_dev(synth.configs.random_images((N, L, L), seed + 2))
        ref = rc.regularize(guide, value, g)
        out = torch.full_like(ref, float("nan"))   # any pixel left unwritten shows
        _noalloc(N, L, patch, window, h, mu, guide, value, g, out)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(out).all())
        assert torch.equal(out, ref), float((out - ref).abs().max())
        rc.close()
