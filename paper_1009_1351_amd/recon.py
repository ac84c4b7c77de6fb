"""Reconstruction context: the Python face of tnlm_recon_init and friends.

Arguments are torch float32 CUDA tensors, contiguous, with the shapes of the
C ABI: images [N][L][L], sinograms [N][V][B]. Work is enqueued on the current
torch stream of the tensors' device.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as nat
from ._native import TnlmError, check


def _ssd_mode(name):
    if name not in nat.SSD_MODES:
        raise ValueError(f"ssd_mode must be one of {sorted(nat.SSD_MODES)}, not {name!r}")
    return nat.SSD_MODES[name]


def _norm_device(device):
    d = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    return torch.device("cuda", torch.cuda.current_device()) if d.index is None else d


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Recon:
    """One slice: geometry (N phases, L x L image, V views, B bins) + parameters."""

    def __init__(self, n_phases, L, n_views, n_bins, view_angles, *, pixel_mm, sad_mm, sdd_mm, dgamma_rad,
                 det_offset_bins=0.25, patch=7, window=15, h=0.007, mu_hat=0.5, beta=1.0, m1=3, m2=1,
                 max_outer=50, tol=0.0, init="fbp", ssd_mode="fp32", device=None):
        self.N, self.L, self.V, self.B = int(n_phases), int(L), int(n_views), int(n_bins)
        self.device = _norm_device(device)
        ang = np.ascontiguousarray(np.asarray(view_angles, dtype=np.float64).reshape(self.N, self.V))
        self._angles = ang
        g = nat.Geometry(self.N, self.L, float(pixel_mm), self.V, self.B, float(sad_mm), float(sdd_mm),
                         float(dgamma_rad), float(det_offset_bins), ang.ctypes.data_as(C.POINTER(C.c_double)))
        p = nat.Params(int(patch), int(window), float(h), float(mu_hat), float(beta), int(m1), int(m2),
                       int(max_outer), float(tol), nat.INIT_FBP_ALL if init == "fbp" else nat.INIT_USER,
                       _ssd_mode(ssd_mode))
        self.params = dict(patch=patch, window=window, h=h, mu_hat=mu_hat, beta=beta, m1=m1, m2=m2,
                           max_outer=max_outer, tol=tol, init=init, ssd_mode=ssd_mode)
        self._ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            check(nat.lib.tnlm_recon_init(C.byref(self._ctx), C.byref(g), C.byref(p),
                                          C.c_void_p(_stream_ptr(self.device))))

    @classmethod
    def from_geometry(cls, geom, **kw):
        """From any object with the ScanGeometry fields (n_phases, L, n_views, ...)."""
        return cls(geom.n_phases, geom.L, geom.n_views, geom.n_bins, geom.view_angles(), pixel_mm=geom.pixel_mm,
                   sad_mm=geom.sad_mm, sdd_mm=geom.sdd_mm, dgamma_rad=geom.dgamma,
                   det_offset_bins=geom.det_offset_bins, **kw)

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            nat.lib.tnlm_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- helpers
    def _img(self, t, name):
        return self._chk(t, (self.N, self.L, self.L), name)

    def _sino(self, t, name):
        return self._chk(t, (self.N, self.V, self.B), name)

    def _chk(self, t, shape, name):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != torch.float32:
            raise TypeError(f"{name} must be a float32 tensor on {self.device}")
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {shape}, got {tuple(t.shape)}")
        return C.c_void_p(t.data_ptr())

    def new_image(self):
        return torch.zeros((self.N, self.L, self.L), dtype=torch.float32, device=self.device)

    def new_sino(self):
        return torch.zeros((self.N, self.V, self.B), dtype=torch.float32, device=self.device)

    # ------------------------------------------------------------ entry points
    def project(self, f, out=None):
        out = self.new_sino() if out is None else out
        check(nat.lib.tnlm_project(self._ctx, self._img(f, "f"), self._sino(out, "q")))
        return out

    def backproject(self, q, out=None):
        out = self.new_image() if out is None else out
        check(nat.lib.tnlm_backproject(self._ctx, self._sino(q, "q"), self._img(out, "f")))
        return out

    def fbp(self, y, all_phases=True, out=None):
        out = self.new_image() if out is None else out
        check(nat.lib.tnlm_fbp(self._ctx, self._sino(y, "y"), self._img(out, "f"), int(bool(all_phases))))
        return out

    def data_step(self, y, w, f, out=None):
        out = self.new_image() if out is None else out
        check(nat.lib.tnlm_data_step(self._ctx, self._sino(y, "y"), self._sino(w, "w"), self._img(f, "f"),
                                     self._img(out, "g")))
        return out

    def regularize(self, guide, value, g, clamp=True, out=None):
        out = self.new_image() if out is None else out
        check(nat.lib.tnlm_regularize(self._ctx, self._img(guide, "guide"), self._img(value, "value"),
                                      self._img(g, "g"), self._img(out, "out"), int(bool(clamp))))
        return out

    def step(self, y, w, f):
        check(nat.lib.tnlm_step(self._ctx, self._sino(y, "y"), self._sino(w, "w"), self._img(f, "f")))
        return f

    def solve(self, y, w, f=None):
        """Returns (f, iterations, last relative update, status)."""
        f = self.new_image() if f is None else f
        iters = C.c_int32(0)
        rel = C.c_float(0.0)
        st = check(nat.lib.tnlm_solve(self._ctx, self._sino(y, "y"), self._sino(w, "w"), self._img(f, "f"),
                                      C.byref(iters), C.byref(rel)))
        return f, iters.value, rel.value, st

    def timing(self, enable: bool):
        check(nat.lib.tnlm_timing_enable(self._ctx, int(bool(enable))))

    def timing_read(self):
        """{kind: (total ms, launches)} since the last read (synchronises)."""
        n = len(nat.KIND_NAMES)
        ms = (C.c_double * n)()
        cnt = (C.c_int32 * n)()
        check(nat.lib.tnlm_timing_read(self._ctx, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(nat.KIND_NAMES)}

    def autotune(self):
        """Pick the regulariser tile height on the device (see tnlm_autotune)."""
        rpl = C.c_int32(0)
        ms = (C.c_float * 2)()
        check(nat.lib.tnlm_autotune(self._ctx, C.byref(rpl), ms))
        return rpl.value, (ms[0], ms[1])

    def cost(self, y, w, f, guide):
        """(data term, regularisation term) of Eq. 1 for f, the weights from
        guide; the cost is data + mu_hat * beta / 2 * reg (tnlm_cost)."""
        data, reg = C.c_double(), C.c_double()
        check(nat.lib.tnlm_cost(self._ctx, self._sino(y, "y"), self._sino(w, "w"), self._img(f, "f"),
                                self._img(guide, "guide"), C.byref(data), C.byref(reg)))
        return data.value, reg.value

    def set_guide(self, guide=None):
        """Fixed weights from `guide` ([N][L][L] float32 on the device) for
        step/solve, or None for the adaptive weights. The tensor must stay
        alive while it is set."""
        self._guide = guide
        check(nat.lib.tnlm_set_guide(self._ctx, None if guide is None else self._img(guide, "guide")))

    def history(self):
        n = self.params["max_outer"]
        buf = (C.c_float * n)()
        cnt = C.c_int32(0)
        check(nat.lib.tnlm_get_history(self._ctx, buf, n, C.byref(cnt)))
        return np.array(buf[:cnt.value], dtype=np.float64)


def _geom_struct(geom, angles_keep):
    ang = np.ascontiguousarray(np.asarray(geom.view_angles(), dtype=np.float64))
    angles_keep.append(ang)
    return nat.Geometry(geom.n_phases, geom.L, float(geom.pixel_mm), geom.n_views, geom.n_bins, float(geom.sad_mm),
                        float(geom.sdd_mm), float(geom.dgamma), float(geom.det_offset_bins),
                        ang.ctypes.data_as(C.POINTER(C.c_double)))


class Batch:
    """Many slices (uneven L, V, B) solved together: tnlm_batch_init / tnlm_batch_solve."""

    def __init__(self, geoms, *, patch=7, window=15, h=0.007, mu_hat=0.5, beta=1.0, m1=3, m2=1, max_outer=50,
                 tol=0.0, init="fbp", ssd_mode="fp32", device=None):
        self.geoms = list(geoms)
        self.device = _norm_device(device)
        self._keep = []
        arr = (nat.Geometry * len(self.geoms))(*[_geom_struct(g, self._keep) for g in self.geoms])
        p = nat.Params(int(patch), int(window), float(h), float(mu_hat), float(beta), int(m1), int(m2),
                       int(max_outer), float(tol), nat.INIT_FBP_ALL if init == "fbp" else nat.INIT_USER,
                       _ssd_mode(ssd_mode))
        self.max_outer = int(max_outer)
        self._b = C.c_void_p()
        with torch.cuda.device(self.device):
            check(nat.lib.tnlm_batch_init(C.byref(self._b), len(self.geoms), arr, C.byref(p),
                                          C.c_void_p(_stream_ptr(self.device))))

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            nat.lib.tnlm_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_images(self):
        return [torch.zeros((g.n_phases, g.L, g.L), dtype=torch.float32, device=self.device) for g in self.geoms]

    def solve(self, ys, ws, fs=None, active=None):
        """Returns (fs, iterations[n], last relative updates[n], statuses[n], worst status).
        active (optional, n booleans): only those slices take part; the others'
        images are left as they are and report 0 iterations."""
        n = len(self.geoms)
        fs = self.new_images() if fs is None else fs
        for g, y, w, f in zip(self.geoms, ys, ws, fs):
            for t, shape in ((y, (g.n_phases, g.n_views, g.n_bins)), (w, (g.n_phases, g.n_views, g.n_bins)),
                             (f, (g.n_phases, g.L, g.L))):
                if t.dtype != torch.float32 or t.device != self.device or tuple(t.shape) != shape \
                        or not t.is_contiguous():
                    raise ValueError(f"batch tensor must be contiguous float32 {shape} on {self.device}")
        P = C.c_void_p * n
        yp = P(*[t.data_ptr() for t in ys])
        wp = P(*[t.data_ptr() for t in ws])
        fp = P(*[t.data_ptr() for t in fs])
        iters = (C.c_int32 * n)()
        rel = (C.c_float * n)()
        sts = (C.c_int * n)()
        if active is None:
            st = nat.lib.tnlm_batch_solve(self._b, yp, wp, fp, iters, rel, sts)
        else:
            if len(active) != n:
                raise ValueError("active needs one entry per slice")
            act = (C.c_int32 * n)(*[1 if a else 0 for a in active])
            st = nat.lib.tnlm_batch_solve_active(self._b, yp, wp, fp, act, iters, rel, sts)
        if st < 0 and all(x >= 0 for x in sts):
            check(st)
        return fs, list(iters), list(rel), list(sts), st

    def timing(self, enable: bool):
        check(nat.lib.tnlm_batch_timing_enable(self._b, int(bool(enable))))

    def timing_read(self):
        k = len(nat.KIND_NAMES)
        ms = (C.c_double * k)()
        cnt = (C.c_int32 * k)()
        check(nat.lib.tnlm_batch_timing_read(self._b, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(nat.KIND_NAMES)}


__all__ = ["Recon", "Batch", "TnlmError"]
