"""Analytic sinograms and the noise model (paper §3, Eq. 9).

Line integrals are computed analytically through each ellipse (no discrete
projector, so the reconstruction's own projector never generates its data).

Noise: the paper adds Gaussian noise of variance exp(p)/N0 (Eq. 9) and uses
the same variance, computed from the noise-free projection p, in the
covariance of the data term. Here the default is the Poisson counting model
the benchmark inputs call for (counts ~ Poisson(I0 exp(-p)), floor at one
count, y = ln(I0 / counts)); ``law="gaussian"`` gives Eq. 9 literally. The
inverse variance handed to the solver is in both cases I0 * exp(-p) computed
from the noise-free p, as in the paper.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import ScanGeometry
from .phantom import Ellipse


def ellipse_line_integrals(src: np.ndarray, u: np.ndarray, ellipses: list[Ellipse]) -> np.ndarray:
    """Sum over ellipses of dmu * chord(ray, ellipse). src, u: [..., 2]."""
    out = np.zeros(src.shape[:-1], dtype=np.float64)
    for e in ellipses:
        c, s = math.cos(e.psi), math.sin(e.psi)
        px, py = src[..., 0] - e.cx, src[..., 1] - e.cy
        qx0 = (px * c + py * s) / e.ax
        qy0 = (-px * s + py * c) / e.ay
        qx1 = (u[..., 0] * c + u[..., 1] * s) / e.ax
        qy1 = (-u[..., 0] * s + u[..., 1] * c) / e.ay
        A = qx1 * qx1 + qy1 * qy1
        Bh = qx0 * qx1 + qy0 * qy1
        C = qx0 * qx0 + qy0 * qy0 - 1.0
        disc = Bh * Bh - A * C
        chord = np.where(disc > 0.0, 2.0 * np.sqrt(np.maximum(disc, 0.0)) / A, 0.0)
        out += e.dmu * chord
    return out


def analytic_sinogram(geom: ScanGeometry, phases: list[list[Ellipse]]) -> np.ndarray:
    """Noise-free [N][V][B] line integrals, phase i from ``phases[i]``."""
    src, u = geom.rays()
    out = np.empty((geom.n_phases, geom.n_views, geom.n_bins), dtype=np.float64)
    for i in range(geom.n_phases):
        out[i] = ellipse_line_integrals(src[i], u[i], phases[i])
    return out


def noisy_measurement(pbar: np.ndarray, I0: float, rng: np.random.Generator, law: str = "poisson"):
    """Returns (y, w): noisy log-projections and inverse variances I0*exp(-pbar)."""
    expected = I0 * np.exp(-pbar)
    if law == "poisson":
        counts = np.maximum(rng.poisson(expected), 1).astype(np.float64)
        y = np.log(I0 / counts)
    elif law == "gaussian":
        y = pbar + rng.standard_normal(pbar.shape) * np.sqrt(np.exp(pbar) / I0)
    elif law == "none":
        y = pbar.copy()
    else:
        raise ValueError(law)
    return y, expected
