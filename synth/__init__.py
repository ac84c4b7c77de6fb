"""Seeded synthetic inputs for the TNLM 4DCT reconstruction.

This package is the "scanner": it builds phantoms, the fan-beam acquisition
geometry (as plain numbers: angles and distances) and noisy sinograms from
analytic ellipse line integrals. It holds none of the reconstruction's
arithmetic (no discrete projector, no CGLS, no patch weights, no FBP), so the
FP64 oracle and the HIP path can both consume what it produces without sharing
any code with each other.
"""
from .geometry import ScanGeometry, paper_scanner
from .phantom import Ellipse, thorax_phantom, rasterize
from .scan import analytic_sinogram, noisy_measurement
from .configs import CONFIGS, make_case, Case

__all__ = [
    "ScanGeometry", "paper_scanner", "Ellipse", "thorax_phantom", "rasterize",
    "analytic_sinogram", "noisy_measurement", "CONFIGS", "make_case", "Case",
]
