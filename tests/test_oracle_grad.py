"""Pins of the oracle's gradient (path-replay adjoint extension).

The oracle's gradient is the exact derivative of its estimator for a fixed
random stream (frozen sampling: collisions decided by the reference medium,
importance-weighted to the evaluated one, majorant held fixed).  It is
pinned by central differences of the oracle's forward pass in that mode, and
statistically by the closed-form Beer-Lambert derivative."""
import dataclasses
import math

import numpy as np
import pytest

import lfsynth as S

from test_oracle_physics import all_rays, chord, homogeneous_scene, ray_geometry


def fd_scene(M=24, spp=6):
    sc = S.config(1, M=M, N=M, spp=spp, max_bounces=3, g=0.3)
    lut = (0.05 + 0.9 * sc.medium.lut).astype(np.float32)  # keep albedo off the clamp kinks
    lut[0, 3] = 0.0
    sc = dataclasses.replace(sc, medium=S.Medium(lut, 25.0),
                             light=dataclasses.replace(sc.light, env=(0.3, 0.2, 0.1)))
    sig = orc_majorant_value(sc)
    return dataclasses.replace(sc, params=dataclasses.replace(sc.params, majorant=sig))


def orc_majorant_value(sc):
    import oracle.oracle as o
    return o.majorant(sc.medium, sc.params)


def test_forward_unchanged_by_frozen_mode_at_theta0(orc):
    sc = fd_scene()
    ks = all_rays(24, 24)[:300]
    a = orc.generate(sc, ks)
    b = orc.generate(sc, ks, sample_medium=S.Medium(sc.medium.lut.copy(), sc.medium.scale))
    assert np.array_equal(a, b)


def test_gradient_matches_central_differences(orc):
    sc = fd_scene()
    rng = np.random.default_rng(8)
    ks = S.random_rays(24, 24, 160, 5)
    adj = rng.standard_normal((len(ks), 3))
    g_lut, g_scale = orc.gradient(sc, ks, adj)
    theta0 = sc.medium

    def loss(lut, scale):
        L = orc.generate(dataclasses.replace(sc, medium=S.Medium(lut, scale)), ks, sample_medium=theta0)
        return float((L * adj).sum())

    touched = np.argwhere(np.abs(g_lut) > 0)
    lut0 = theta0.lut

    def central(h):
        fd = np.zeros_like(g_lut)
        for e, c in touched:
            lp, lm = lut0.copy(), lut0.copy()
            lp[e, c] += h
            lm[e, c] -= h
            step = float(lp[e, c]) - float(lm[e, c])  # the FP32 table holds the rounded step
            fd[e, c] = (loss(lp, theta0.scale) - loss(lm, theta0.scale)) / step
        return fd

    # the estimator is smooth in theta: the central-difference error falls as
    # h^2 (measured 1.7e-2, 1.5e-3, 1.7e-4, 1.5e-5 at h = 1e-2 .. 3e-4)
    err3 = np.linalg.norm(central(1e-3) - g_lut) / np.linalg.norm(g_lut)
    err4 = np.linalg.norm(central(3e-4) - g_lut) / np.linalg.norm(g_lut)
    assert err3 < 1e-3 and err4 < 5e-5 and err4 < err3 / 5, (err3, err4)
    h = 1e-4
    fd_s = (loss(lut0, theta0.scale + h) - loss(lut0, theta0.scale - h)) / (2 * h)
    # untouched entries have zero derivative: perturbing one changes nothing
    for e, c in [(200, 3), (128, 0)]:
        if g_lut[e, c] == 0:
            lp = lut0.copy()
            lp[e, c] += h
            assert loss(lp, theta0.scale) == loss(lut0, theta0.scale)
    assert len(touched) > 100
    assert abs(fd_s - g_scale) < 1e-4 * abs(g_scale)


def test_gradient_beer_lambert_closed_form(orc):
    """Homogeneous absorber, albedo 0, env 1: E[dLhat/dscale] = -alpha l e^{-sigma l}
    and E[dLhat/dLUT[1].alpha] = -scale l e^{-sigma l} (the constant volume
    maps to the last LUT entry), with sigma = scale * alpha."""
    alpha, scale = 0.1, 10.0
    sc = homogeneous_scene(M=24, spp=4096, alpha=alpha, scale=scale)
    sigma = alpha * scale
    ks = all_rays(24, 24)[::7]
    geo = ray_geometry(orc, 24, 24, ks)
    ell = np.array([chord(o, d)[0] for o, d in geo])
    p = np.exp(-sigma * ell)
    adj = np.zeros((len(ks), 3))
    adj[:, 0] = 1.0
    g_lut, g_scale = orc.gradient(sc, ks, adj)
    expect = -(alpha * ell * p).sum()
    sbar = 1.25 * sigma
    # per sample: transmitted (prob p) times the null-collision score sum,
    # whose variance is alpha^2 l / (sbar - sigma); second moment bound
    var = (p * (alpha ** 2 * ell / (sbar - sigma) + (alpha * ell) ** 2)).sum() / 4096
    assert abs(g_scale - expect) < 5 * math.sqrt(var)
    # the trilinear weights sum to 1 only up to rounding, so entry 0 gets ~1e-15
    assert abs(g_lut[0, 3]) < 1e-9 * abs(g_lut[1, 3]) and np.all(g_lut[:, :3] == 0.0)
    expect_a = -(scale * ell * p).sum()
    var_a = (p * (scale ** 2 * ell / (sbar - sigma) + (scale * ell) ** 2)).sum() / 4096
    assert abs(g_lut[1, 3] - expect_a) < 5 * math.sqrt(var_a)


def test_gradient_albedo_single_scatter(orc):
    """With one scatter vertex every NEE contribution is linear in the albedo,
    so d/d rgb of the LUT equals the radiance divided by the albedo."""
    rgb = (0.7, 0.5, 0.3)
    sc = homogeneous_scene(M=16, spp=64, alpha=0.1, rgb=rgb, env=(0, 0, 0), radiance=(1.0, 1.0, 1.0),
                           max_bounces=1)
    ks = all_rays(16, 16)
    L = orc.generate(sc, ks)
    adj = np.ones((len(ks), 3))
    g_lut, _ = orc.gradient(sc, ks, adj)
    # the constant volume uses entry 1 only (w = 1)
    for c in range(3):
        rho = float(np.float32(rgb[c]))  # the LUT is stored in binary32
        assert abs(g_lut[1, c] - L[:, c].sum() / rho) < 1e-9 * L[:, c].sum()
        assert abs(g_lut[0, c]) < 1e-12 * abs(g_lut[1, c])
