"""Pins of the oracle's mean SSIM (Wang et al. 2004), the image index the
paper reports for its light-field views against path-traced references."""
import math

import numpy as np
import pytest
from scipy import ndimage


def gaussian11():
    g = np.exp(-((np.arange(11) - 5) ** 2) / (2 * 1.5 ** 2))
    return g / g.sum()


def ssim_separable(a, b, rng_=1.0):
    """The same index through scipy's separable correlation (an independent
    implementation: 1-D passes, 'valid' crop)."""
    g = gaussian11()
    c1, c2 = (0.01 * rng_) ** 2, (0.03 * rng_) ** 2
    out = []
    for x, y in zip(a.astype(np.float64), b.astype(np.float64)):
        vals = []
        for c in range(3):
            X, Y = x[..., c], y[..., c]

            def f(z):
                z = ndimage.correlate1d(z, g, axis=0, mode="constant")
                z = ndimage.correlate1d(z, g, axis=1, mode="constant")
                return z[5:-5, 5:-5]
            mx, my = f(X), f(Y)
            sx, sy, sxy = f(X * X) - mx * mx, f(Y * Y) - my * my, f(X * Y) - mx * my
            vals.append(((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sx + sy + c2)))
        out.append(np.mean(vals))
    return np.array(out)


def test_ssim_identity_and_symmetry(orc):
    rng = np.random.default_rng(1)
    a = rng.uniform(0, 1, (2, 23, 31, 3)).astype(np.float32)
    b = np.clip(a + rng.normal(0, 0.1, a.shape), 0, 1).astype(np.float32)
    assert np.allclose(orc.ssim(a, a), 1.0, atol=1e-12)
    assert np.allclose(orc.ssim(a, b), orc.ssim(b, a), atol=1e-14)
    assert np.all(orc.ssim(a, b) < 0.99)


def test_ssim_constant_images_closed_form(orc):
    for p, q in ((0.2, 0.7), (0.5, 0.5), (0.9, 0.1)):
        a = np.full((1, 16, 20, 3), p, np.float32)
        b = np.full((1, 16, 20, 3), q, np.float32)
        pf, qf = float(np.float32(p)), float(np.float32(q))
        c1 = 1e-4
        expect = (2 * pf * qf + c1) / (pf * pf + qf * qf + c1)
        assert abs(orc.ssim(a, b)[0] - expect) < 1e-12


def test_ssim_matches_separable_filter(orc):
    rng = np.random.default_rng(2)
    a = rng.uniform(0, 1, (3, 30, 26, 3)).astype(np.float32)
    smooth = ndimage.gaussian_filter(a, sigma=(0, 2, 2, 0))
    b = (0.7 * smooth + 0.3 * rng.uniform(0, 1, a.shape)).astype(np.float32)
    got = orc.ssim(a, b, 1.0)
    ref = ssim_separable(a, b, 1.0)
    assert np.abs(got - ref).max() < 1e-12
    assert np.abs(orc.ssim(a, b, 2.5) - ssim_separable(a, b, 2.5)).max() < 1e-12
