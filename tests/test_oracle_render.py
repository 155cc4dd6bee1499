"""Pins of the oracle's ground-truth views (the path tracer of Sec. 2 along
pinhole camera rays; the paper compares its light-field views against such
path-traced references in its evaluation).

Expected values come from closed forms computed here with the test's own
camera geometry and slab clipping, and from the light-field rays of the same
lines (whose estimator is pinned in test_oracle_physics.py)."""
import dataclasses
import math

import numpy as np
import pytest

import lfsynth as S

from test_oracle_lookup import line_camera
from test_oracle_physics import chord, homogeneous_scene


def pixel_dir(cam, W, H, x, y):
    f = np.subtract(cam.target, cam.eye)
    f = f / np.linalg.norm(f)
    r = np.cross(f, cam.up)
    r = r / np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(0.5 * cam.vfov)
    d = f + (2 * (x + 0.5) / W - 1) * th * W / H * r + (1 - 2 * (y + 0.5) / H) * th * u
    return d / np.linalg.norm(d)


def test_render_vacuum_is_environment(orc):
    sc = homogeneous_scene(scale=0.0, env=(0.2, 0.5, 1.0), radiance=(1.0, 1.0, 1.0), spp=4)
    cams = S.cameras(5, 2, math.sqrt(3.0))
    pix = orc.all_pixels(2, 12, 9)
    rgb = orc.render(sc, cams, 12, 9, pix)
    assert np.all(rgb == np.array([0.2, 0.5, 1.0]))


def test_render_beer_lambert_along_camera_rays(orc):
    spp = 4096
    sc = homogeneous_scene(spp=spp, alpha=0.1, scale=10.0)   # sigma = 1, albedo 0, env 1
    cams = S.cameras(6, 2, math.sqrt(3.0))
    W, H = 10, 8
    pix = orc.all_pixels(2, W, H)
    rgb = orc.render(sc, cams, W, H, pix)
    p = np.array([math.exp(-chord(np.array(cams[v].eye), pixel_dir(cams[v], W, H, x, y))[0])
                  for v, x, y in pix])
    assert np.all(rgb[:, 0] == rgb[:, 2])
    sd = np.sqrt(p * (1 - p) / spp)
    assert np.all(np.abs(rgb[:, 0] - p) <= 5.5 * sd + 1e-12)
    assert (p < 0.999).sum() > 40 and (p == 1.0).sum() > 5  # pixels through and beside the box
    z = (rgb[:, 0] - p).sum() / math.sqrt((sd ** 2).sum() + 1e-300)
    assert abs(z) < 5


def test_render_matches_light_field_rays_in_expectation(orc):
    """A pixel whose ray is the line of light-field ray (i, j), jitter off:
    both estimate the radiance along that line (8 seeds each, scattering
    scene with next-event estimation and the majorant grid)."""
    M = N = 64
    base = S.config(1, M=M, N=N, spp=512, max_bounces=4, g=0.3, jitter=0)
    base = dataclasses.replace(base, medium=S.Medium(base.medium.lut, 60.0),
                               light=dataclasses.replace(base.light, radiance=(4.0, 4.0, 4.0),
                                                         env=(0.1, 0.1, 0.1)))
    pairs = [(3, 40), (17, 50), (30, 9), (45, 21), (60, 2)]
    W, H = 9, 7
    cams = [line_camera(orc, M, N, i, j, W, H) for i, j in pairs]
    pix = np.array([[v, W // 2, H // 2] for v in range(len(pairs))], np.int32)
    ks = np.array([i * N + j for i, j in pairs])
    a, b = [], []
    for seed in range(8):
        sc = base.with_params(seed=500 + seed)
        a.append(orc.render(sc, cams, W, H, pix))
        b.append(orc.generate(sc, ks))
    a, b = np.array(a), np.array(b)
    diff = a.mean(0) - b.mean(0)
    se = np.sqrt(a.var(0, ddof=1) / 8 + b.var(0, ddof=1) / 8) + 1e-12
    assert np.abs(diff / se).max() < 6.0
    # the medium matters on these lines: attenuation and in-scattered light
    assert np.abs(b.mean(0) - 0.1).max() > 0.05 and (b.mean(0) > 0.1).any()
