"""FP64 CPU oracle (test infrastructure).

ctypes front-end of ``oracle_tnlm.c``. Only the test-suite, the smoke check
and the benchmark's CPU-baseline leg use this package; the HIP library never
imports, links or calls it. It takes the plain numbers of an acquisition
(``synth.ScanGeometry``-like objects: phases, L, views, bins, distances and
view angles) and NumPy float64 arrays.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle_tnlm.so")
_SRC = os.path.join(_HERE, "oracle_tnlm.c")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (C, FP64, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


@contextlib.contextmanager
def _lib_threads(n: int):
    """Run the oracle's OpenMP loops on n threads inside the block."""
    L = lib()
    prev = L.omp_get_max_threads()
    L.omp_set_num_threads(int(n))
    try:
        yield
    finally:
        L.omp_set_num_threads(prev)


class _Geom(C.Structure):
    _fields_ = [("n_phases", C.c_int32), ("L", C.c_int32), ("pixel_mm", C.c_double),
                ("n_views", C.c_int32), ("n_bins", C.c_int32), ("sad_mm", C.c_double),
                ("sdd_mm", C.c_double), ("dgamma_rad", C.c_double), ("det_offset_bins", C.c_double),
                ("view_angles", C.POINTER(C.c_double))]


class _Params(C.Structure):
    _fields_ = [("patch", C.c_int32), ("window", C.c_int32), ("h", C.c_double), ("mu_hat", C.c_double),
                ("beta", C.c_double), ("m1_cgls", C.c_int32), ("m2_jacobi", C.c_int32),
                ("max_outer", C.c_int32), ("tol_rel_update", C.c_double),
                ("guide", C.POINTER(C.c_double))]   # NULL: weights from g^(k); else fixed weights (Eq. 3)


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        D = C.POINTER(C.c_double)
        G = C.POINTER(_Geom)
        P = C.POINTER(_Params)
        for name, args, res in [
            ("orc_project", [G, D, D], None),
            ("orc_backproject", [G, D, D], None),
            ("orc_trace_ray", [G, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int32), D], C.c_int),
            ("orc_fbp", [G, D, D, C.c_int], None),
            ("orc_cgls", [G, D, D, D, C.c_int, C.c_double, D], None),
            ("orc_weights", [C.c_int, C.c_int, C.c_int, C.c_double, D, D, C.c_int, C.c_int, D, D], None),
            ("orc_regularize", [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, D, D, D, D,
                                C.c_int], None),
            ("orc_gauss_jacobi", [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, D, D, D],
             None),
            ("orc_step", [G, P, D, D, D], C.c_double),
            ("orc_solve", [G, P, D, D, D, C.c_int, D, D], C.c_int),
            ("orc_cost", [G, P, D, D, D, D, D, D], None),
            ("orc_power_beta", [G, D, C.c_int], C.c_double),
        ]:
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = res
    return _lib


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _arr(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Geometry:
    """Holds the C geometry struct plus the arrays it points to."""

    def __init__(self, geom):
        self.src = geom
        self.N, self.L, self.V, self.B = geom.n_phases, geom.L, geom.n_views, geom.n_bins
        self.angles = _arr(geom.view_angles())
        self.c = _Geom(geom.n_phases, geom.L, geom.pixel_mm, geom.n_views, geom.n_bins, geom.sad_mm,
                       geom.sdd_mm, geom.dgamma, geom.det_offset_bins, _d(self.angles))

    def ref(self):
        return C.byref(self.c)


def _geom(g) -> Geometry:
    return g if isinstance(g, Geometry) else Geometry(g)


def params(patch=5, window=11, h=0.02, mu_hat=1.0, beta=1.0, m1=3, m2=1, max_outer=10, tol=0.0,
           guide=None) -> _Params:
    """guide: None, or an [N][L][L] stack from which the weights are taken in
    every outer iteration instead of from the data-step output (Eq. 3 with a
    fixed image, e.g. the ground truth)."""
    p = _Params(patch, window, h, mu_hat, beta, m1, m2, max_outer, tol, None)
    if guide is not None:
        p._guide = np.ascontiguousarray(guide, dtype=np.float64)   # kept alive with the struct
        p.guide = _d(p._guide)
    return p


def case_params(case, **over) -> _Params:
    kw = dict(patch=case.patch, window=case.window, h=case.h, mu_hat=case.mu_hat, beta=case.beta,
              m1=case.m1, m2=case.m2, max_outer=case.max_outer, tol=case.tol)
    kw.update(over)
    return params(**kw)


def project(geom, f) -> np.ndarray:
    g = _geom(geom)
    f = _arr(f).reshape(g.N, g.L, g.L)
    q = np.empty((g.N, g.V, g.B))
    lib().orc_project(g.ref(), _d(f), _d(q))
    return q


def backproject(geom, q) -> np.ndarray:
    g = _geom(geom)
    q = _arr(q).reshape(g.N, g.V, g.B)
    f = np.empty((g.N, g.L, g.L))
    lib().orc_backproject(g.ref(), _d(q), _d(f))
    return f


def trace_ray(geom, i, v, b):
    g = _geom(geom)
    pix = np.empty(4 * g.L + 8, dtype=np.int32)
    ln = np.empty(4 * g.L + 8)
    n = lib().orc_trace_ray(g.ref(), i, v, b, pix.ctypes.data_as(C.POINTER(C.c_int32)), _d(ln))
    return pix[:n].copy(), ln[:n].copy()


def fbp(geom, y, all_phases=True) -> np.ndarray:
    g = _geom(geom)
    y = _arr(y).reshape(g.N, g.V, g.B)
    f = np.empty((g.N, g.L, g.L))
    lib().orc_fbp(g.ref(), _d(y), _d(f), int(bool(all_phases)))
    return f


def cgls(geom, y, w, f, m1=3, beta=1.0) -> np.ndarray:
    g = _geom(geom)
    y, w, f = _arr(y), _arr(w), _arr(f)
    out = np.empty((g.N, g.L, g.L))
    lib().orc_cgls(g.ref(), _d(y), _d(w), _d(f), int(m1), float(beta), _d(out))
    return out


def weights(gi, gj, r, c, patch, window, h):
    gi, gj = _arr(gi), _arr(gj)
    L = gi.shape[-1]
    w = np.empty(window * window)
    dist = np.empty(window * window)
    lib().orc_weights(L, patch, window, h, _d(gi), _d(gj), r, c, _d(w), _d(dist))
    return w.reshape(window, window), dist.reshape(window, window)


def regularize(guide, value, g, patch, window, h, mu_hat, clamp=True) -> np.ndarray:
    guide, value, g = _arr(guide), _arr(value), _arr(g)
    N, L = g.shape[0], g.shape[-1]
    out = np.empty_like(g)
    lib().orc_regularize(N, L, patch, window, h, mu_hat, _d(guide), _d(value), _d(g), _d(out), int(bool(clamp)))
    return out


def gauss_jacobi(g, patch, window, h, mu_hat, m2=1, guide=None) -> np.ndarray:
    g = _arr(g)
    N, L = g.shape[0], g.shape[-1]
    out = np.empty_like(g)
    gd = None if guide is None else _arr(guide)
    lib().orc_gauss_jacobi(N, L, patch, window, h, mu_hat, m2, _d(g), None if gd is None else _d(gd), _d(out))
    return out


def step(geom, prm, y, w, f):
    """One outer iteration; returns (f_new, relative update)."""
    g = _geom(geom)
    f = _arr(f).copy()
    rel = lib().orc_step(g.ref(), C.byref(prm), _d(_arr(y)), _d(_arr(w)), _d(f))
    return f, rel


def solve(geom, prm, y, w, f0=None):
    """Full solve; returns (f, iterations, last relative update, history)."""
    g = _geom(geom)
    f = np.zeros((g.N, g.L, g.L)) if f0 is None else _arr(f0).copy()
    rel = C.c_double(0.0)
    hist = np.zeros(max(prm.max_outer, 1))
    k = lib().orc_solve(g.ref(), C.byref(prm), _d(_arr(y)), _d(_arr(w)), _d(f), int(f0 is None),
                        C.byref(rel), _d(hist))
    return f, k, rel.value, hist[:k].copy()


def cost(geom, prm, y, w, f, guide):
    """(data term, sum of J terms); total cost = data + mu_hat*beta/2 * reg (Eq. 1)."""
    g = _geom(geom)
    data, reg = C.c_double(), C.c_double()
    lib().orc_cost(g.ref(), C.byref(prm), _d(_arr(y)), _d(_arr(w)), _d(_arr(f)), _d(_arr(guide)),
                   C.byref(data), C.byref(reg))
    return data.value, reg.value


def power_beta(geom, w, iters=30) -> float:
    """Largest eigenvalue of P^T S^-1 P (max over phases), by power iteration."""
    g = _geom(geom)
    return lib().orc_power_beta(g.ref(), _d(_arr(w)), int(iters))
