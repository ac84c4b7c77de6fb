"""Coarse-to-fine start of the TNLM solve (the multi-grid speed-up that §4
proposes; Python face of tnlm_image_upsample plus the batch engine).

Each slice is first solved on the grid with half the side -- pixels twice as
large over the same field, the same views, bins and measured data -- to a
looser relative-update tolerance, for at most coarse_max iterations (a coarse
solve that settles into the period-2 cycle of the outer iteration stops
there); the bilinear upsampling of that solution is the start of the solve
at full resolution. As with the learned start, a slice that stalls at full
resolution (warmstart.StartedSolver's check) or is still above the tolerance
after `restart_after` iterations restarts from the FBP of all phases. All
arithmetic runs in the library's kernels; this module orchestrates.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import torch

from . import _native as nat
from ._native import check_cnn
from .recon import Batch, _norm_device


def upsample(images, factor=2, out=None):
    """Bilinear upsampling of a [n][h][w] float32 device tensor by `factor`."""
    n, h, w = images.shape
    if images.dtype != torch.float32 or not images.is_contiguous() or images.device.type != "cuda":
        raise ValueError("images must be a contiguous float32 CUDA tensor [n][h][w]")
    out = torch.empty((n, h * factor, w * factor), dtype=torch.float32, device=images.device) if out is None else out
    with torch.cuda.device(images.device):
        stream = torch.cuda.current_stream(images.device).cuda_stream
        check_cnn(nat.lib.tnlm_image_upsample(C.c_void_p(images.data_ptr()), C.c_void_p(out.data_ptr()), n, h, w,
                                              int(factor), C.c_void_p(stream)))
    return out


def coarse_geometry(geom):
    """The same scan on a grid with half the side (L must be even)."""
    if geom.L % 2:
        raise ValueError("the image side must be even for a coarse level")
    return dataclasses.replace(geom, L=geom.L // 2)


class MultigridSolver:
    """Coarse-to-fine solve of a fixed set of slice geometries to a
    relative-update tolerance (contexts built once, at construction): the
    coarse level batched, then StartedSolver at full resolution from the
    upsampled coarse images (batched, stall check, cold restart).
    solve() returns (images, full-resolution iterations, coarse iterations,
    statuses); the full-resolution count includes a cold restart's."""

    def __init__(self, geoms, *, patch, window, h, mu_hat, tol, max_outer, coarse_tol=1e-3, coarse_max=50,
                 restart_after=None, stall_window=10, stall_ratio=0.6, device=None):
        from .warmstart import StartedSolver
        self.device = _norm_device(device)
        self.n = len(geoms)
        kw = dict(patch=patch, window=window, h=h, mu_hat=mu_hat, device=self.device)
        self.coarse = Batch([coarse_geometry(g) for g in geoms], init="fbp", max_outer=coarse_max, tol=coarse_tol,
                            **kw)
        self.fine = StartedSolver(geoms, tol=tol, max_outer=max_outer, restart_after=restart_after,
                                  stall_window=stall_window, stall_ratio=stall_ratio, **kw)

    def solve(self, ys, ws):
        fc, itc, _, _, _ = self.coarse.solve(ys, ws)
        f0 = [upsample(f) for f in fc]
        fs, iters, st = self.fine.solve(ys, ws, f0)
        return fs, iters, list(itc), st

    def close(self):
        self.coarse.close()
        self.fine.close()


__all__ = ["upsample", "coarse_geometry", "MultigridSolver"]
