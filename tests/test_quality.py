"""Pins of the image-quality measures (Eqs. 10 and 11) and of the regions of
interest built on the phantom (CPU)."""
import math

import numpy as np
import pytest

import synth
from synth import quality


@pytest.mark.parametrize("config", ["C1", "C2c"])
def test_regions_are_pure_and_disjoint(config):
    case = synth.make_case(config)
    for i, els in enumerate(case.ellipses):
        rg = quality.regions(els, case.geom.L, case.geom.fov_mm)
        for sig, bg in rg.values():
            assert sig.sum() > 0 and bg.sum() > 0 and not (sig & bg).any()
        # the phantom is constant inside each region: tumour / lung, vertebra / tissue
        t = case.truth[i]
        (s1, b1), (s2, b2) = rg["roi1"], rg["roi2"]
        for m in (s1, b1, s2, b2):
            assert np.ptp(t[m]) < 1e-12
        assert t[s1][0] > t[b1][0] and t[s2][0] > t[b2][0]


def test_cnr_of_a_constructed_image():
    img = np.zeros((8, 8))
    sig = np.zeros((8, 8), bool)
    sig[:2] = True
    bg = np.zeros((8, 8), bool)
    bg[4:] = True
    img[sig] = 5.0
    img[4:] = np.where(np.arange(8) % 2 == 0, 1.5, 0.5)[None, :]   # mean 1, population std 0.5
    assert quality.cnr(img, sig, bg) == pytest.approx(8.0, abs=1e-12)


def test_snr_definition_properties():
    rng = np.random.default_rng(3)
    truth = rng.uniform(0, 1, size=(16, 16))
    assert quality.snr(truth, truth) == math.inf
    noisy = truth + rng.normal(0, 0.05, size=truth.shape)
    assert quality.snr(3.0 * noisy, 3.0 * truth) == pytest.approx(quality.snr(noisy, truth), abs=1e-9)
    # the numerator is taken about the image's own mean: a constant offset of the
    # truth changes only the error term
    off = truth + 0.1
    expect = 10 * math.log10(np.sum((off - off.mean()) ** 2) / (0.01 * off.size))
    assert quality.snr(off, truth) == pytest.approx(expect, rel=1e-12)
    # halving the error raises the SNR by 10 log10(4) dB when the image is fixed
    half = truth + 0.5 * (noisy - truth)
    assert quality.snr(noisy, half) - quality.snr(noisy, truth) == pytest.approx(10 * math.log10(4.0), abs=1e-9)
