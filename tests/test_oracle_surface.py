"""Pins of the oracle's isosurface variant (the paper renders segmented
surfaces): first crossing of the trilinear field through the isovalue,
Lambertian shading with next-event estimation, cosine-weighted bounces."""
import dataclasses
import math

import numpy as np
import pytest

import lfsynth as S

from test_oracle_render import pixel_dir

R0 = 0.6


def sphere_volume(n=64):
    """f = R0 - |p| at the voxel centres: the isosurface f = 0 is close to the
    sphere of radius R0 (trilinear interpolation of a cone)."""
    idx = (np.arange(n) + 0.5) / n * 2 - 1
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    f = (R0 - np.sqrt(x * x + y * y + z * z)).astype(np.float32)
    return S.Volume(f.reshape(-1), S.F32, (n, n, n), 0, -1.0, 1.0)


def surface_scene(rgb=(1.0, 1.0, 1.0), env=(1.0, 1.0, 1.0), radiance=(0.0, 0.0, 0.0), max_bounces=64, spp=8,
                  vol=None, iso=0.0):
    lut = S.constant_lut(rgb, 0.5)
    light = S.Light(kind=S.DIRECTIONAL, dir=tuple(np.array([0.2, 0.4, 0.9]) / np.linalg.norm([0.2, 0.4, 0.9])),
                    radiance=radiance, env=env)
    prm = S.Params(M=32, N=32, spp=spp, max_bounces=max_bounces, seed=31, jitter=1, surface=1, iso=iso)
    return S.Scene("surf", vol or sphere_volume(), S.Medium(lut, 1.0), light, prm)


def test_surface_hit_sphere_distance(orc):
    sc = surface_scene()
    rng = np.random.default_rng(3)
    for _ in range(60):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        x = -2.5 * d + 0.2 * rng.uniform(-1, 1) * np.cross(d, [0.3, 0.5, 0.8])
        b = float(np.dot(x, d))
        c = float(np.dot(x, x)) - R0 * R0
        disc = b * b - c
        t = orc.surface_hit(sc.volume, sc.params, x, d, 0.0, 6.0)
        if disc > 0.02:
            assert t is not None and abs(t - (-b - math.sqrt(disc))) < 4e-3
        elif disc < -0.02:
            assert t is None


def test_surface_hit_is_the_first_crossing(orc):
    """On the phantom: the returned point lies on the isosurface (to the
    bisection's width) and no earlier half-voxel sample changes sign."""
    sc = S.config(2, vol_n=64)
    iso = 1024.0 - 500.0   # between air (-1000 HU) and the body (-100..300 HU)
    prm = dataclasses.replace(sc.params, surface=1, iso=iso)
    vol = sc.volume
    h = 0.5 * 2.0 / 64
    rng = np.random.default_rng(4)
    hits = 0
    for _ in range(40):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        x = -3.0 * d + 0.3 * rng.standard_normal(3)
        t0, t1 = 1.0, 5.0
        t = orc.surface_hit(vol, prm, x, d, t0, t1)
        ts = t0 + h * np.arange(int((t1 - t0) / h) + 1)
        # the oracle's own field at the samples (sigma_at of an identity LUT is the raw value)
        raw = raw_at(orc, vol, x[None, :] + ts[:, None] * d[None, :])
        sgn = raw - iso >= 0
        change = np.nonzero(sgn[1:] != sgn[:-1])[0]
        if t is None:
            assert len(change) == 0
            continue
        hits += 1
        m = change[0]
        assert ts[m] <= t <= ts[m + 1] + 1e-12
        fr = raw_at(orc, vol, (x + t * d)[None, :])[0]
        assert abs(fr - iso) < 1e-6 * 3000
    assert hits > 10


def raw_at(orc, vol, pts):
    """Raw trilinear value: sigma_at with a LUT whose alpha is the window
    position, times the window width."""
    lut = np.zeros((2, 4), np.float32)
    lut[1, 3] = 1.0
    s = orc.sigma_at(vol, S.Medium(lut, 1.0), pts)
    return vol.vmin + s * (vol.vmax - vol.vmin)


def test_surface_white_furnace(orc):
    """Albedo 1 under a uniform environment: every sample returns exactly
    the environment (energy conservation; the phantom's surface is not
    convex)."""
    sc = surface_scene()
    L = orc.generate(sc, np.arange(32 * 32)[(np.arange(32 * 32) // 32) != (np.arange(32 * 32) % 32)])
    assert np.all(L == 1.0)
    ph = S.config(2, vol_n=64)
    sc2 = surface_scene(vol=ph.volume, iso=1024.0 - 500.0, max_bounces=200)
    ks = np.arange(0, 32 * 32, 7)
    ks = ks[(ks // 32) != (ks % 32)]   # texels i == j are 0 by definition
    L2, st = orc.generate(sc2, ks, stats=True)
    assert np.all(L2 == 1.0) and st[2] > 100


def test_surface_direct_lighting_closed_form(orc):
    """One vertex, directional light E, black environment: a pixel that hits
    the sphere is rho / pi * max(0, n . w) * E with n the sphere normal at
    the analytic hit (the convex sphere never shadows its lit side)."""
    rho = 0.6
    sc = surface_scene(rgb=(rho, rho, rho), env=(0.0, 0.0, 0.0), radiance=(2.0, 2.0, 2.0), max_bounces=1, spp=2)
    w = np.array(sc.light.dir)
    cams = S.cameras(9, 2, math.sqrt(3.0))
    W, H = 32, 24
    pix = orc.all_pixels(2, W, H)
    rgb = orc.render(sc, cams, W, H, pix)
    n_hit = 0
    for (v, x, y), val in zip(pix, rgb):
        eye = np.array(cams[v].eye)
        d = pixel_dir(cams[v], W, H, x, y)
        b = float(np.dot(eye, d))
        disc = b * b - (float(np.dot(eye, eye)) - R0 * R0)
        if disc < 0.02:
            if disc < -0.02:
                assert np.all(val == 0.0)
            continue
        p = eye + (-b - math.sqrt(disc)) * d
        expect = rho / math.pi * max(0.0, float(np.dot(p / R0, w))) * 2.0
        assert abs(val[0] - expect) < 0.02 * rho * 2.0 / math.pi, (val, expect)
        n_hit += 1
    assert n_hit > 80
