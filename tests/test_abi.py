"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tnlm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tnlm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ["tnlm_recon_init", "tnlm_step", "tnlm_solve", "tnlm_destroy", "tnlm_project",
                 "tnlm_backproject", "tnlm_fbp", "tnlm_data_step", "tnlm_regularize"]:
        assert name in fns


def test_library_exports_every_declared_symbol():
    from paper_1009_1351_amd import _native
    for name in declared_functions():
        assert hasattr(_native.lib, name), name
        assert name in _native.exported_symbols()


def _geom_params(**over):
    from paper_1009_1351_amd import _native as nat
    ang = np.zeros((2, 4))
    g = dict(n_phases=2, L=16, pixel_mm=10.0, n_views=4, n_bins=8, sad_mm=541.0, sdd_mm=949.075,
             dgamma_rad=0.01, det_offset_bins=0.25)
    p = dict(patch=3, window=5, h=0.01, mu_hat=0.5, beta=1.0, m1_cgls=3, m2_jacobi=1, max_outer=2,
             tol_rel_update=0.0, init=0, ssd_mode=0)
    for k, v in over.items():
        (g if k in g else p)[k] = v
    G = nat.Geometry(g["n_phases"], g["L"], g["pixel_mm"], g["n_views"], g["n_bins"], g["sad_mm"], g["sdd_mm"],
                     g["dgamma_rad"], g["det_offset_bins"], ang.ctypes.data_as(C.POINTER(C.c_double)))
    P = nat.Params(*[p[k] for k in ["patch", "window", "h", "mu_hat", "beta", "m1_cgls", "m2_jacobi", "max_outer",
                                   "tol_rel_update", "init", "ssd_mode"]])
    return G, P, ang


@pytest.mark.parametrize("over,code", [
    (dict(patch=4), -1), (dict(window=6), -1), (dict(window=17), -2), (dict(h=0.0), -1),
    (dict(mu_hat=-1.0), -1), (dict(beta=0.0), -1), (dict(m2_jacobi=0), -1), (dict(max_outer=0), -1),
    (dict(n_phases=0), -2), (dict(L=0), -2), (dict(n_bins=0), -2), (dict(pixel_mm=-1.0), -1),
    (dict(sad_mm=10.0), -1), (dict(init=7), -1), (dict(tol_rel_update=-1.0), -1), (dict(ssd_mode=3), -1),
    (dict(L=32, patch=9, window=21, ssd_mode=2), -1),   # symmetric reuse: window 21 exceeds a block's LDS
])
def test_init_rejects_bad_arguments(over, code):
    from paper_1009_1351_amd import _native as nat
    G, P, _ang = _geom_params(**over)
    ctx = C.c_void_p(123)
    st = nat.lib.tnlm_recon_init(C.byref(ctx), C.byref(G), C.byref(P), None)
    assert st == code
    assert ctx.value is None
    assert len(nat.lib.tnlm_last_error()) > 0


def test_entry_points_reject_null_context():
    from paper_1009_1351_amd import _native as nat
    assert nat.lib.tnlm_step(None, None, None, None) == -1
    assert nat.lib.tnlm_project(None, None, None) == -1
    assert nat.lib.tnlm_status_string(-5) == b"non-finite value"
    assert nat.lib.tnlm_cost(None, None, None, None, None, None, None) == -1
    assert nat.lib.tnlm_batch_solve_active(None, None, None, None, None, None, None, None) == -1


def test_nonfinite_view_angle_rejected():
    from paper_1009_1351_amd import _native as nat
    G, P, ang = _geom_params()
    ang[1, 2] = np.nan
    ctx = C.c_void_p()
    assert nat.lib.tnlm_recon_init(C.byref(ctx), C.byref(G), C.byref(P), None) == -5


def test_noalloc_regulariser_rejects_bad_arguments():
    """tnlm_regularize_noalloc checks its arguments before any HIP call."""
    from paper_1009_1351_amd import _native as nat
    f = nat.lib.tnlm_regularize_noalloc
    a, b, c, d = C.c_void_p(16), C.c_void_p(32), C.c_void_p(48), C.c_void_p(64)
    assert f(2, 16, 3, 5, 0.01, 0.5, None, b, c, d, 1, None) == -1          # null input
    assert f(2, 16, 3, 5, 0.01, 0.5, a, b, c, a, 1, None) == -1             # output aliases an input
    assert f(2, 5000, 3, 5, 0.01, 0.5, a, b, c, d, 1, None) == -2           # L beyond 4096
    assert f(0, 16, 3, 5, 0.01, 0.5, a, b, c, d, 1, None) == -2             # no phase
    assert f(200, 4096, 3, 5, 0.01, 0.5, a, b, c, d, 1, None) == -2         # N L^2 beyond 2^31
    assert f(2, 16, 4, 5, 0.01, 0.5, a, b, c, d, 1, None) == -1             # even patch
    assert f(2, 4, 3, 5, 0.01, 0.5, a, b, c, d, 1, None) == -2              # window beyond the image
    assert f(2, 16, 3, 5, 0.0, 0.5, a, b, c, d, 1, None) == -1              # h = 0
    assert f(2, 16, 3, 5, 0.01, -1.0, a, b, c, d, 1, None) == -1            # mu_hat < 0
    assert b"4096" in nat.lib.tnlm_last_error() or len(nat.lib.tnlm_last_error()) > 0
