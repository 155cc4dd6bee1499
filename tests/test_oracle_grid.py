"""Pins of the oracle's majorant grid (piecewise-constant majorant of delta
and ratio tracking).

A majorant grid changes which tentative points are drawn but not what the
estimator converges to, so it is pinned by:
  - brute force: sigma_t sampled densely, also up to one voxel outside each
    cell, never exceeds the cell's majorant / 1.25;
  - closed forms: a constant volume, the floor in empty space;
  - quadrature: heterogeneous transmittance exp(-integral of sigma_t) of a
    pure absorber (sigma_t sampled along the chord, not tracked);
  - expectation: scattering scenes with shadow rays agree with the global
    majorant within their statistical error;
  - identity: where every cell's majorant equals the global one, the walk
    through the cells reproduces the global-majorant result to rounding;
  - central differences of the frozen-sampling estimator for the gradient.
"""
import dataclasses
import math

import numpy as np
import pytest

import lfsynth as S

from test_oracle_physics import chord, ray_geometry


def box_points(rng, n, lo=-1.0, hi=1.0):
    return rng.uniform(lo, hi, (n, 3))


def cell_of(pts, G, lo=-1.0, hi=1.0):
    c = np.floor((pts - lo) / (hi - lo) * G).astype(np.int64)
    return np.clip(c, 0, G - 1)


@pytest.mark.parametrize("c,G,vol_n", [(1, 8, None), (1, 7, None), (2, 16, 64), (5, 5, 32)])
def test_grid_bounds_sigma(orc, c, G, vol_n):
    sc = S.config(c, vol_n=vol_n) if vol_n else S.config(c)
    prm = dataclasses.replace(sc.params, grid=G)
    maj = orc.majorant_grid(sc.volume, sc.medium, prm)
    rng = np.random.default_rng(20 + c)
    pts = box_points(rng, 120_000)
    n = sc.volume.dims[0]
    h = 2.0 / n
    cells = cell_of(pts, G)
    m = maj[cells[:, 2], cells[:, 1], cells[:, 0]]
    sig = orc.sigma_at(sc.volume, sc.medium, pts)
    assert np.all(1.25 * sig <= m * (1 + 1e-12))
    # up to one voxel outside the cell (rounding of the cell a point falls in)
    moved = np.clip(pts + rng.uniform(-0.95 * h, 0.95 * h, pts.shape), -1.0, 1.0)
    sig2 = orc.sigma_at(sc.volume, sc.medium, moved)
    assert np.all(1.25 * sig2 <= m * (1 + 1e-12))
    glob = orc.majorant(sc.medium, sc.params)
    assert np.all(maj <= glob * (1 + 1e-12)) and np.all(maj >= glob / 256 * (1 - 1e-12))
    # the grid is much tighter than the global majorant on these volumes
    assert maj.mean() < 0.6 * glob


def test_grid_constant_volume_closed_form(orc):
    lut = np.zeros((5, 4), np.float32)
    lut[:, 3] = [0.0, 0.2, 0.9, 0.4, 0.1]
    lut[:, :3] = 0.5
    for value, (e0, e1) in ((0.3, (1, 2)), (0.5, (2, 3)), (1.0, (3, 4)), (0.0, (0, 1))):
        vol = S.constant_volume(8, value)
        prm = S.Params(M=4, N=4, grid=3)
        maj = orc.majorant_grid(vol, S.Medium(lut, 2.0), prm)
        expect = max(1.25 * 2.0 * float(max(lut[e0, 3], lut[e1, 3])), 1.25 * 2.0 * 0.9 / 256)
        assert np.allclose(maj, expect, rtol=1e-15, atol=0), (value, maj.ravel()[:3], expect)


def test_grid_floor_in_empty_space(orc):
    sc = S.config(1)
    lut = sc.medium.lut.copy()
    lut[: lut.shape[0] // 2, 3] = 0.0  # transparent below half of the window
    med = S.Medium(lut, sc.medium.scale)
    maj = orc.majorant_grid(sc.volume, med, dataclasses.replace(sc.params, grid=8))
    glob = orc.majorant(med, sc.params)
    # cells near the box corners hold only low values: exactly the floor
    assert maj[0, 0, 0] == glob / 256 and maj[-1, -1, -1] == glob / 256
    assert (maj == glob / 256).sum() > 50 and (maj > glob / 256).sum() > 20


def absorber_scene(G, spp, jitter=0):
    sc = S.config(1, M=24, N=24, spp=spp, max_bounces=4, grid=G, jitter=jitter)
    lut = sc.medium.lut.copy()
    lut[:, :3] = 0.0  # albedo 0: the first real collision ends the sample
    return dataclasses.replace(sc, medium=S.Medium(lut, 30.0),
                               light=dataclasses.replace(sc.light, radiance=(0.0, 0.0, 0.0),
                                                         env=(1.0, 1.0, 1.0)))


@pytest.mark.parametrize("G", [0, 8, 13])
def test_grid_transmittance_quadrature(orc, G):
    """Pure absorber, environment 1: each sample is 1 with probability
    exp(-integral of sigma_t along the chord)."""
    spp = 4096
    sc = absorber_scene(G, spp)
    ks = S.random_rays(24, 24, 48, 3)
    L = orc.generate(sc, ks)[:, 0]
    p = []
    for o, d in ray_geometry(orc, 24, 24, ks):
        ell, t0, t1 = chord(o, d)
        if ell == 0.0:
            p.append(1.0)
            continue
        m = 6000
        ts = t0 + (np.arange(m) + 0.5) * (ell / m)
        sig = orc.sigma_at(sc.volume, sc.medium, o[None, :] + ts[:, None] * d[None, :])
        p.append(math.exp(-sig.sum() * ell / m))
    p = np.array(p)
    sd = np.sqrt(p * (1 - p) / spp)
    assert np.all(np.abs(L - p) <= 5.5 * sd + 1e-6)
    z = (L - p).sum() / math.sqrt((sd ** 2).sum())
    assert abs(z) < 5
    assert 0.05 < p.mean() < 0.95  # the medium is neither vacuum nor opaque


def test_grid_agrees_with_global_majorant_in_expectation(orc):
    """Scattering blob scene with a directional light (free flights and
    shadow rays both walk the grid): mean radiance per ray over 8 seeds
    agrees with the global-majorant estimator within its error."""
    base = S.config(1, M=16, N=16, spp=256, max_bounces=4, g=0.3, jitter=1)
    base = dataclasses.replace(base, medium=S.Medium(base.medium.lut, 60.0),
                               light=dataclasses.replace(base.light, radiance=(4.0, 4.0, 4.0)))
    ks = S.random_rays(16, 16, 40, 4)
    runs = {0: [], 8: []}
    for G in runs:
        for seed in range(8):
            sc = base.with_params(grid=G, seed=900 + seed)
            runs[G].append(orc.generate(sc, ks))
    a, b = np.array(runs[0]), np.array(runs[8])          # [seed, ray, 3]
    diff = a.mean(0) - b.mean(0)
    se = np.sqrt(a.var(0, ddof=1) / 8 + b.var(0, ddof=1) / 8) + 1e-12
    t = diff / se
    assert np.abs(t).max() < 6.5
    assert abs(diff.sum() / math.sqrt((se ** 2).sum())) < 5
    assert a.mean() > 0.01  # light reaches the rays (the environment is black: NEE only)


def test_grid_identity_when_cells_match_global(orc):
    """A LUT of constant alpha gives every cell the global majorant: walking
    the cells spends the same optical depth as the single global segment, so
    the results agree to rounding."""
    sc = S.config(1, M=16, N=16, spp=32, max_bounces=4, g=0.3, jitter=1)
    lut = sc.medium.lut.copy()
    lut[:, 3] = 0.4
    sc = dataclasses.replace(sc, medium=S.Medium(lut, 6.0))
    ks = np.arange(16 * 16)
    ks = ks[(ks // 16) != (ks % 16)]
    a, st_a = orc.generate(sc, ks, stats=True)
    b, st_b = orc.generate(sc.with_params(grid=8), ks, stats=True)
    maj = orc.majorant_grid(sc.volume, sc.medium, sc.params.__class__(**{**sc.params.__dict__, "grid": 8}))
    assert np.all(maj == orc.majorant(sc.medium, sc.params))
    assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(a).max())
    assert np.array_equal(st_a, st_b)


def test_grid_gradient_matches_central_differences(orc):
    """Frozen sampling with the grid built from the reference medium: the
    path-replay gradient is the derivative of the estimator."""
    sc = S.config(1, M=20, N=20, spp=6, max_bounces=3, g=0.3, grid=8)
    lut = (0.05 + 0.9 * sc.medium.lut).astype(np.float32)
    lut[0, 3] = 0.0
    sc = dataclasses.replace(sc, medium=S.Medium(lut, 25.0),
                             light=dataclasses.replace(sc.light, env=(0.3, 0.2, 0.1)))
    rng = np.random.default_rng(18)
    ks = S.random_rays(20, 20, 120, 6)
    adj = rng.standard_normal((len(ks), 3))
    g_lut, g_scale = orc.gradient(sc, ks, adj)
    theta0 = sc.medium

    def loss(lut_, scale):
        L = orc.generate(dataclasses.replace(sc, medium=S.Medium(lut_, scale)), ks, sample_medium=theta0)
        return float((L * adj).sum())

    touched = np.argwhere(np.abs(g_lut) > 1e-9 * np.abs(g_lut).max())
    h = 3e-4
    fd = np.zeros_like(g_lut)
    for e, c in touched:
        lp, lm = lut.copy(), lut.copy()
        lp[e, c] += h
        lm[e, c] -= h
        fd[e, c] = (loss(lp, theta0.scale) - loss(lm, theta0.scale)) / (float(lp[e, c]) - float(lm[e, c]))
    err = np.linalg.norm(fd - g_lut) / np.linalg.norm(g_lut)
    assert err < 5e-5, err
    fd_s = (loss(lut, theta0.scale + 1e-4) - loss(lut, theta0.scale - 1e-4)) / 2e-4
    assert abs(fd_s - g_scale) < 1e-4 * abs(g_scale)
    assert len(touched) > 100
