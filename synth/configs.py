"""Benchmark workload definitions (sizes, doses, seeds) and case construction.

Workloads, all 10 phases per slice on the paper's scanner geometry:
  C1  1 slice, 64^2, 90 views, 96 bins, I0 1e4, patch 5, window 11, 10 its
  C2  1 slice, 256^2, 512 bins, patch 7, window 15, 50 its, three dose cases
      a: 360 views at I0 2e4 (all projections, low dose: paper Case 1)
      b: 60 views at I0 1e6 (under-sampled, high dose: paper Case 2)
      c: 60 views at I0 2e4 (under-sampled, low dose: paper Case 3)
  C3  64 slices, L from {128,256,384,512}, V from [40,360], I0 log-uniform
      [1e4,1e6], B = 1.5 L, patch 7, window 15
  C4  32 slices, 512^2, 720 bins, 120 views, I0 5e4, patch 7, window 15
  C5  learned warm start: train at 256^2 (512 bins, 60 views, I0 log-uniform
      [1e4,1e5]); evaluate 32 slices at 512^2, 720 bins, 60 views, I0 2e4,
      to relative update 1e-4

Seeds: phantom of slice s uses PCG64(10091351 + s); the noise of (slice s,
phase i) uses PCG64(10091351 + 10**6 + 1000 s + i).

The regularisation strength h is expressed relative to the patch size and the
image scale: h^2 = h_rel^2 * d^2 * (0.01 / mm)^2, so one value of h_rel serves
every patch size. The default (0.1) comes from a sweep of the FP64 oracle on
C1 (relative L2 error to the phantom after K iterations, which is flat over
h_rel in [0.05, 0.6] there). The workloads that run to a relative-update
tolerance (C5) use 0.6, the smallest value of a sweep at which most 256^2 and
512^2 slices converge instead of oscillating between two states.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .geometry import ScanGeometry
from .phantom import thorax_phantom, rasterize
from .scan import analytic_sinogram, noisy_measurement

SEED = 10091351
H_REL_DEFAULT = 0.1
# Workloads that stop on the relative update use a larger h: at h_rel <= 0.4
# the outer iteration of many 256^2 and 512^2 slices settles into a period-2
# oscillation (relative update ~1e-3 forever); at 0.6 most slices converge.
H_REL_TO_TOL = 0.6
MU_HAT_DEFAULT = 0.5


def h_from_rel(h_rel: float, patch: int) -> float:
    return h_rel * patch * 0.01


@dataclasses.dataclass
class Case:
    name: str
    geom: ScanGeometry
    y: np.ndarray       # [N][V][B] float64
    w: np.ndarray       # [N][V][B] float64, inverse variance
    I0: float
    patch: int
    window: int
    h: float
    mu_hat: float
    beta: float
    m1: int
    m2: int
    max_outer: int
    tol: float
    ellipses: list = None   # per phase: the phantom's ellipses (for regions of interest)
    _truth: np.ndarray = dataclasses.field(default=None, repr=False)

    @property
    def truth(self) -> np.ndarray:
        """[N][L][L] float64 phantom (4x4 supersampled), rasterised on first use."""
        if self._truth is None:
            L = self.geom.L
            self._truth = np.stack([rasterize(el, L, self.geom.fov_mm) for el in self.ellipses])
        return self._truth


CONFIGS = {
    "C1": dict(L=64, V=90, B=96, I0=1e4, patch=5, window=11, K=10, tol=0.0),
    "C2a": dict(L=256, V=360, B=512, I0=2e4, patch=7, window=15, K=50, tol=0.0),
    "C2b": dict(L=256, V=60, B=512, I0=1e6, patch=7, window=15, K=50, tol=0.0),
    "C2c": dict(L=256, V=60, B=512, I0=2e4, patch=7, window=15, K=50, tol=0.0),
    "C4": dict(L=512, V=120, B=720, I0=5e4, patch=7, window=15, K=50, tol=0.0),
    "C5train": dict(L=256, V=60, B=512, I0=None, patch=7, window=15, K=600, tol=1e-4, h_rel=H_REL_TO_TOL),
    "C5eval": dict(L=512, V=60, B=720, I0=2e4, patch=7, window=15, K=600, tol=1e-4, h_rel=H_REL_TO_TOL),
}


def c3_slice_shape(s: int):
    """(L, V, B, I0) of slice s of the 64-slice mixed batch."""
    rng = np.random.Generator(np.random.PCG64(SEED + 7 * 10**6 + s))
    L = int(rng.choice([128, 256, 384, 512]))
    V = int(rng.integers(40, 361))
    I0 = float(10.0 ** rng.uniform(4.0, 6.0))
    return L, V, int(round(1.5 * L)), I0


def make_case(config: str = "C1", slice_index: int = 0, n_phases: int = 10, *, L=None, V=None, B=None,
              I0=None, patch=None, window=None, K=None, tol=None, h_rel=None,
              mu_hat=MU_HAT_DEFAULT, m1=3, m2=1, beta=1.0, randomize=None, law="poisson") -> Case:
    if config == "C3":
        L0, V0, B0, I00 = c3_slice_shape(slice_index)
        base = dict(L=L0, V=V0, B=B0, I0=I00, patch=7, window=15, K=50, tol=0.0)
    else:
        base = dict(CONFIGS[config])
    L = L if L is not None else base["L"]
    V = V if V is not None else base["V"]
    B = B if B is not None else base["B"]
    patch = patch if patch is not None else base["patch"]
    window = window if window is not None else base["window"]
    K = K if K is not None else base["K"]
    tol = tol if tol is not None else base["tol"]
    h_rel = h_rel if h_rel is not None else base.get("h_rel", H_REL_DEFAULT)
    if I0 is None:
        I0 = base["I0"]
    if I0 is None:  # C5 training: log-uniform dose around the evaluation dose
        r = np.random.Generator(np.random.PCG64(SEED + 5 * 10**6 + slice_index))
        I0 = float(10.0 ** r.uniform(4.0, 5.0))
    if randomize is None:
        randomize = config in ("C3", "C5train", "C5eval", "C4")
    geom = ScanGeometry(n_phases=n_phases, L=L, n_views=V, n_bins=B)
    phases = []
    for i in range(n_phases):
        rng = np.random.Generator(np.random.PCG64(SEED + slice_index))  # same draws for every phase
        phases.append(thorax_phantom(i, n_phases, geom.pixel_mm, rng=rng, randomize=randomize))
    pbar = analytic_sinogram(geom, phases)
    y = np.empty_like(pbar)
    w = np.empty_like(pbar)
    for i in range(n_phases):
        rng = np.random.Generator(np.random.PCG64(SEED + 10**6 + 1000 * slice_index + i))
        y[i], w[i] = noisy_measurement(pbar[i], I0, rng, law=law)
    return Case(name=f"{config}/s{slice_index}", geom=geom, y=y, w=w, I0=I0, patch=patch,
                window=window, h=h_from_rel(h_rel, patch), mu_hat=mu_hat, beta=beta, m1=m1, m2=m2,
                max_outer=K, tol=tol, ellipses=phases)


def random_images(shape, seed: int, lo: float = 0.0, hi: float = 0.03) -> np.ndarray:
    """Uniform random test images (for operator-level parity and pins)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=shape)


def smooth_random_images(shape, seed: int, scale: float = 0.02, passes: int = 2) -> np.ndarray:
    """Random images smoothed by a few 3x3 box passes (patch-structured content)."""
    a = random_images(shape, seed, 0.0, 1.0)
    for _ in range(passes):
        p = np.pad(a, [(0, 0)] * (a.ndim - 2) + [(1, 1), (1, 1)], mode="edge")
        a = sum(p[..., dy:dy + shape[-2], dx:dx + shape[-1]] for dy in range(3) for dx in range(3)) / 9.0
    return a * scale


def angles_for(geom: ScanGeometry) -> np.ndarray:
    return geom.view_angles()


__all__ = ["Case", "CONFIGS", "make_case", "c3_slice_shape", "random_images", "smooth_random_images",
           "h_from_rel"]
