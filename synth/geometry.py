"""Fan-beam arc-detector acquisition geometry (paper §3, first paragraph).

The scanner of the paper's experiments: an arc detector of 888 units at
1.0239 mm pitch, source-to-detector distance 949.075 mm, source-to-rotation-
centre distance 541.0 mm. The detector's angular extent (fan angle) follows
from those numbers: 888 * 1.0239 / 949.075 rad.

Conventions shared by every consumer (stated here once, as numbers):
  * image: L x L pixels covering a square of side ``fov_mm`` centred on the
    rotation axis; row index r grows along +y, column index c along +x;
    pixel (r, c) centre = ((c + 1/2) * D - S/2, (r + 1/2) * D - S/2), D = S/L.
  * view angle theta: source at SAD * (cos theta, sin theta).
  * bin b of B: fan angle gamma_b = (b - (B-1)/2 + det_offset) * dgamma;
    the ray leaves the source with direction angle theta + pi + gamma_b.
  * phase i of N, view v of V: theta = theta0 + 2*pi*(v + i/N)/V, so the
    union of all phases' views is N*V uniformly interleaved views.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Scanner constants printed in the paper (§3, experimental set-up).
PAPER_DET_UNITS = 888
PAPER_DET_PITCH_MM = 1.0239
PAPER_SDD_MM = 949.075
PAPER_SAD_MM = 541.0
FAN_ANGLE_RAD = PAPER_DET_UNITS * PAPER_DET_PITCH_MM / PAPER_SDD_MM


@dataclasses.dataclass(frozen=True)
class ScanGeometry:
    n_phases: int
    L: int
    n_views: int
    n_bins: int
    fov_mm: float = 500.0
    sad_mm: float = PAPER_SAD_MM
    sdd_mm: float = PAPER_SDD_MM
    det_offset_bins: float = 0.25
    theta0: float = 0.0

    @property
    def pixel_mm(self) -> float:
        return self.fov_mm / self.L

    @property
    def dgamma(self) -> float:
        return FAN_ANGLE_RAD / self.n_bins

    def view_angles(self) -> np.ndarray:
        """[N][V] view angles in radians (float64)."""
        i = np.arange(self.n_phases, dtype=np.float64)[:, None]
        v = np.arange(self.n_views, dtype=np.float64)[None, :]
        return self.theta0 + 2.0 * math.pi * (v + i / self.n_phases) / self.n_views

    def fan_angles(self) -> np.ndarray:
        b = np.arange(self.n_bins, dtype=np.float64)
        return (b - (self.n_bins - 1) / 2.0 + self.det_offset_bins) * self.dgamma

    def rays(self):
        """Source points and unit directions, each [N][V][B][2] float64."""
        th = self.view_angles()[:, :, None]
        g = self.fan_angles()[None, None, :]
        src = np.stack(np.broadcast_arrays(self.sad_mm * np.cos(th), self.sad_mm * np.sin(th)), -1)
        src = np.broadcast_to(src, th.shape[:2] + (self.n_bins, 2))
        phi = th + math.pi + g
        u = np.stack([np.cos(phi), np.sin(phi)], -1)
        return np.ascontiguousarray(src), u


def paper_scanner(n_phases: int, L: int, n_views: int, n_bins: int, **kw) -> ScanGeometry:
    return ScanGeometry(n_phases=n_phases, L=L, n_views=n_views, n_bins=n_bins, **kw)
