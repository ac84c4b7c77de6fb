"""Nested-ellipse thorax phantom with a moving 'tumour' (stand-in for NCAT).

The paper evaluates on the NCAT thorax phantom, which is not available; this
family keeps its role (a breathing thorax slice, 10 phases, a small
high-contrast structure moving inside the lung) with an own, simple design.

Ellipses are listed in painter's order (each one sits entirely inside the one
it overrides), so the attenuation map is the *sum* of per-ellipse increments
``mu_k - mu_parent``. That additive form is what makes analytic line
integrals exact.

Units: millimetres and attenuation per millimetre (0 .. 0.03 / mm).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Ellipse:
    cx: float
    cy: float
    ax: float      # semi-axis along the ellipse's own x
    ay: float      # semi-axis along the ellipse's own y
    psi: float     # rotation (rad)
    dmu: float     # additive attenuation increment (1/mm)


def _tumour_shift_px(i: int, n: int, amp_px: float, phase0: float) -> float:
    # displacement along -y: amp/2 * (1 - cos(2 pi (i/N + phase0))) pixels;
    # amp = 8 px gives 0 .. 8 px with the largest step between consecutive
    # phases 2.47 px, inside every search window used here.
    return 0.5 * amp_px * (1.0 - math.cos(2.0 * math.pi * (i / n + phase0)))


def thorax_phantom(phase: int, n_phases: int, pixel_mm: float, rng: np.random.Generator | None = None,
                   randomize: bool = False) -> list[Ellipse]:
    """Ellipses of one respiratory phase.

    With ``randomize`` the slice-level shape parameters are drawn from ``rng``
    (axes +-10 %, attenuations +-5 %, tumour radius / position / amplitude /
    phase offset); pass the same generator state for every phase of a slice.
    """
    body_a, body_b = 170.0, 120.0
    lung_a, lung_b = 45.0, 80.0
    mu_body, mu_lung, mu_heart, mu_bone, mu_tum = 0.019, 0.004, 0.021, 0.030, 0.020
    heart_r, bone_r, tum_r = 35.0, 18.0, 9.0
    tum_x, tum_y = 80.0, 45.0
    amp_px, phase0 = 8.0, 0.0
    if randomize:
        assert rng is not None
        s = lambda: 1.0 + rng.uniform(-0.10, 0.10)   # noqa: E731
        m = lambda: 1.0 + rng.uniform(-0.05, 0.05)   # noqa: E731
        body_a, body_b = body_a * s(), body_b * s()
        lung_a, lung_b = lung_a * s(), lung_b * s()
        heart_r, bone_r = heart_r * s(), bone_r * s()
        mu_body, mu_lung, mu_heart, mu_bone, mu_tum = (mu_body * m(), mu_lung * m(), mu_heart * m(),
                                                       mu_bone * m(), mu_tum * m())
        tum_r = rng.uniform(6.0, 12.0)
        tum_x = 80.0 + rng.uniform(-10.0, 10.0)
        tum_y = 40.0 + rng.uniform(-10.0, 10.0)
        amp_px = rng.uniform(0.0, 8.0)
        phase0 = rng.uniform(0.0, 1.0)
    # keep the tumour (with its largest displacement) inside the right lung
    shift_mm = _tumour_shift_px(phase, n_phases, amp_px, phase0) * pixel_mm
    shift_mm = min(shift_mm, 0.6 * lung_b)
    lung_cy = 10.0
    return [
        Ellipse(0.0, 0.0, body_a, body_b, 0.0, mu_body),
        Ellipse(+80.0, lung_cy, lung_a, lung_b, 0.0, mu_lung - mu_body),
        Ellipse(-80.0, lung_cy, lung_a, lung_b, 0.0, mu_lung - mu_body),
        Ellipse(0.0, 30.0, heart_r, heart_r, 0.0, mu_heart - mu_body),
        Ellipse(0.0, -85.0, bone_r, bone_r, 0.0, mu_bone - mu_body),
        Ellipse(tum_x, tum_y - shift_mm, tum_r, tum_r, 0.0, mu_tum - mu_lung),
    ]


def rasterize(ellipses: list[Ellipse], L: int, fov_mm: float = 500.0, supersample: int = 4) -> np.ndarray:
    """[L][L] image (row along +y), each pixel the mean over ss x ss sub-samples.

    Each ellipse is tested only on the sub-samples of its bounding square
    (radius = its larger semi-axis); the others receive nothing from it, so
    the result equals the test over the whole grid."""
    D = fov_mm / L
    n = L * supersample
    k = (np.arange(n, dtype=np.float64) + 0.5) * (D / supersample) - fov_mm / 2.0
    img = np.zeros((n, n))
    for e in ellipses:
        c, s = math.cos(e.psi), math.sin(e.psi)
        rad = max(e.ax, e.ay)
        cols = np.nonzero(np.abs(k - e.cx) <= rad)[0]
        rows = np.nonzero(np.abs(k - e.cy) <= rad)[0]
        if cols.size == 0 or rows.size == 0:
            continue
        c0, c1, r0, r1 = cols[0], cols[-1] + 1, rows[0], rows[-1] + 1
        X, Y = np.meshgrid(k[c0:c1], k[r0:r1])   # Y varies along rows
        xr = (X - e.cx) * c + (Y - e.cy) * s
        yr = -(X - e.cx) * s + (Y - e.cy) * c
        img[r0:r1, c0:c1] += np.where((xr / e.ax) ** 2 + (yr / e.ay) ** 2 <= 1.0, e.dmu, 0.0)
    return img.reshape(L, supersample, L, supersample).mean(axis=(1, 3))
