"""Image-quality measures of §3 on the synthetic phantom: contrast-to-noise
ratio on a region of interest (Eq. 10) and signal-to-noise ratio against the
ground truth (Eq. 11), with the two regions of the paper's evaluation
rebuilt on this phantom: a small high-contrast structure against the lung
around it (the tumour), and the vertebral body against the soft tissue
around it. Regions come from each phase's ellipses, shrunk (signal) or kept
clear of edges (background) so partial-volume pixels do not enter.
"""
from __future__ import annotations

import math

import numpy as np

from .phantom import Ellipse


def _inside(e: Ellipse, scale: float, L: int, fov_mm: float) -> np.ndarray:
    """Pixels whose centre lies inside ellipse e with its axes scaled by `scale`."""
    D = fov_mm / L
    k = (np.arange(L) + 0.5) * D - fov_mm / 2.0
    X, Y = np.meshgrid(k, k)
    c, s = math.cos(e.psi), math.sin(e.psi)
    xr = (X - e.cx) * c + (Y - e.cy) * s
    yr = -(X - e.cx) * s + (Y - e.cy) * c
    return (xr / (e.ax * scale)) ** 2 + (yr / (e.ay * scale)) ** 2 <= 1.0


def _near(e: Ellipse, radius_factor: float, L: int, fov_mm: float) -> np.ndarray:
    return _inside(Ellipse(e.cx, e.cy, e.ax, e.ay, e.psi, 0.0), radius_factor, L, fov_mm)


def regions(ellipses: list[Ellipse], L: int, fov_mm: float = 500.0) -> dict:
    """(signal, background) masks of the two regions for one phase.

    Ellipses in the order of thorax_phantom: body, lung at +x (with the
    tumour), lung at -x, heart, vertebra, tumour."""
    body, lung_r, lung_l, heart, bone, tum = ellipses
    lungs = _inside(lung_r, 1.0, L, fov_mm) | _inside(lung_l, 1.0, L, fov_mm)
    roi1_sig = _inside(tum, 0.6, L, fov_mm)
    roi1_bg = (_inside(lung_r, 0.9, L, fov_mm) & ~_near(tum, 1.6, L, fov_mm) & _near(tum, 3.0, L, fov_mm))
    roi2_sig = _inside(bone, 0.6, L, fov_mm)
    roi2_bg = (_inside(body, 0.95, L, fov_mm) & ~_near(bone, 1.6, L, fov_mm) & _near(bone, 3.0, L, fov_mm)
               & ~_near(lung_r, 1.1, L, fov_mm) & ~_near(lung_l, 1.1, L, fov_mm) & ~_near(heart, 1.1, L, fov_mm)
               & ~lungs)
    return {"roi1": (roi1_sig, roi1_bg), "roi2": (roi2_sig, roi2_bg)}


def cnr(img: np.ndarray, signal: np.ndarray, background: np.ndarray) -> float:
    """Eq. 10: |mean(signal) - mean(background)| / std(background) (population std)."""
    b = img[background]
    return float(abs(img[signal].mean() - b.mean()) / b.std())


def snr(img: np.ndarray, truth: np.ndarray) -> float:
    """Eq. 11: 10 log10(||f - mean(f)||^2 / ||f - f*||^2), in dB."""
    num = float(np.sum((img - img.mean()) ** 2))
    den = float(np.sum((img - truth) ** 2))
    return math.inf if den == 0.0 else 10.0 * math.log10(num / den)


def report(stack: np.ndarray, case) -> dict:
    """Means over the phases of a reconstruction [N][L][L] of `case`, as in
    the paper's tables: CNR of both regions and SNR."""
    L = case.geom.L
    c1, c2, sn = [], [], []
    for i, els in enumerate(case.ellipses):
        rg = regions(els, L, case.geom.fov_mm)
        c1.append(cnr(stack[i], *rg["roi1"]))
        c2.append(cnr(stack[i], *rg["roi2"]))
        sn.append(snr(stack[i], case.truth[i]))
    return {"cnr_roi1": float(np.mean(c1)), "cnr_roi2": float(np.mean(c2)), "snr_db": float(np.mean(sn))}


__all__ = ["regions", "cnr", "snr", "report"]
