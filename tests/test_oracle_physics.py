"""Physics pins of the oracle's light-field generation (Sec. 2: ray set R^K,
origin jitter, path tracer -- read volumetrically).

Expected values come from closed forms and quadrature computed here with
the test's own geometry (slab clipping, Gauss-Legendre), not from the
oracle's code: Beer-Lambert transmittance, white-furnace energy
conservation, vacuum, linearity, and single scattering under a directional
and an area light."""
import dataclasses
import math

import numpy as np
import pytest

import lfsynth as S


def homogeneous_scene(M=48, spp=256, alpha=0.1, rgb=(0.0, 0.0, 0.0), scale=10.0, env=(1.0, 1.0, 1.0),
                      radiance=(0.0, 0.0, 0.0), max_bounces=4, g=0.0, jitter=0, light=None, majorant=0.0):
    vol = S.constant_volume(8, 1.0)
    med = S.Medium(S.constant_lut(rgb, alpha), scale)
    lt = light or S.Light(kind=S.DIRECTIONAL, dir=tuple(np.array([0.3, 0.5, 0.81]) / np.linalg.norm([0.3, 0.5, 0.81])))
    lt = dataclasses.replace(lt, radiance=radiance, env=env)
    prm = S.Params(M=M, N=M, spp=spp, max_bounces=max_bounces, g=g, seed=77, jitter=jitter, majorant=majorant)
    return S.Scene("homog", vol, med, lt, prm)


def chord(o, d, lo=-1.0, hi=1.0):
    """Length of the ray o + t d (t >= 0) inside the box [lo, hi]^3."""
    t0, t1 = 0.0, math.inf
    for a in range(3):
        if d[a] == 0:
            if not lo <= o[a] <= hi:
                return 0.0, 0.0, 0.0
            continue
        ta, tb = (lo - o[a]) / d[a], (hi - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return (t1 - t0, t0, t1) if t1 > t0 else (0.0, 0.0, 0.0)


def ray_geometry(orc, M, N, ks, R=math.sqrt(3.0)):
    Po, Pd = orc.sf_points(M), orc.sf_points(N)
    out = []
    for k in ks:
        i, j = divmod(int(k), N)
        d = Pd[j] - Po[i]
        out.append((R * Po[i], d / np.linalg.norm(d)))
    return out


def all_rays(M, N):
    k = np.arange(M * N)
    return k[(k // N) != (k % N)]


@pytest.mark.parametrize("majorant", [0.0, 1.0, 4.0])
def test_beer_lambert(orc, majorant):
    sc = homogeneous_scene(majorant=majorant)
    sigma = 10.0 * 0.1
    ks = all_rays(48, 48)
    L = orc.generate(sc, ks)
    p = np.array([math.exp(-sigma * chord(o, d)[0]) for o, d in ray_geometry(orc, 48, 48, ks)])
    spp = sc.params.spp
    # each sample is 1 (transmitted) or 0 (absorbed): binomial bounds
    assert np.all(L[:, 0] == L[:, 1]) and np.all(L[:, 0] == L[:, 2])
    assert np.all(np.abs(L[:, 0] - p) <= 5.5 * np.sqrt(p * (1 - p) / spp) + 1e-12)
    z = (L[:, 0] - p).sum() / math.sqrt((p * (1 - p) / spp).sum())
    assert abs(z) < 5
    assert abs(L[:, 0].mean() - p.mean()) < 1e-3


def test_beer_lambert_jittered_disk(orc):
    """Origins uniform on the disk of area 4 pi R^2 / M (radius 2R/sqrt(M)) in
    the tangent plane: the expectation is the disk average of exp(-sigma l)."""
    M = 12
    sc = homogeneous_scene(M=M, spp=8192, jitter=1)
    sigma = 1.0
    ks = np.array([0 * M + 5, 3 * M + 7, 6 * M + 1, 9 * M + 2, 11 * M + 4])
    L = orc.generate(sc, ks)
    R = math.sqrt(3.0)
    rad = 2 * R / math.sqrt(M)
    xr, wr = np.polynomial.legendre.leggauss(48)
    for (o, d), Lk in zip(ray_geometry(orc, M, M, ks), L[:, 0]):
        n = o / np.linalg.norm(o)
        t1 = np.cross(n, [0.3, 0.1, 0.9])
        t1 /= np.linalg.norm(t1)
        t2 = np.cross(n, t1)
        acc = 0.0
        for x, w in zip(xr, wr):  # r in [0, rad], area measure r dr dtheta
            r = 0.5 * rad * (x + 1)
            for th in np.linspace(0, 2 * math.pi, 96, endpoint=False):
                oo = o + r * (math.cos(th) * t1 + math.sin(th) * t2)
                acc += w * 0.5 * rad * r * (2 * math.pi / 96) * math.exp(-sigma * chord(oo, d)[0])
        p = acc / (math.pi * rad * rad)
        assert abs(Lk - p) <= 5 * math.sqrt(p * (1 - p) / 8192) + 1e-9
    # without jitter the same rays give a different (unblurred) answer
    L0 = orc.generate(dataclasses.replace(sc, params=dataclasses.replace(sc.params, jitter=0)), ks)
    assert np.abs(L0 - L).max() > 0.01


@pytest.mark.parametrize("g", [0.0, 0.3])
def test_white_furnace_homogeneous(orc, g):
    sc = homogeneous_scene(alpha=0.2, rgb=(1.0, 1.0, 1.0), max_bounces=1000, g=g, jitter=1, spp=32)
    L = orc.generate(sc, all_rays(48, 48))
    assert np.all(L == 1.0)


def test_white_furnace_heterogeneous(orc):
    """Energy conservation in the c1 blob volume with albedo 1: every sample
    returns exactly the environment radiance 1."""
    sc = S.config(1, M=64, N=64, spp=8, max_bounces=1000)
    lut = sc.medium.lut.copy()
    lut[:, :3] = 1.0
    sc = dataclasses.replace(sc, medium=S.Medium(lut, 40.0),
                             light=dataclasses.replace(sc.light, radiance=(0, 0, 0), env=(1.0, 1.0, 1.0)))
    L, st = orc.generate(sc, all_rays(64, 64), stats=True)
    assert np.all(L == 1.0)
    assert st[2] > 1000  # many real collisions were involved


def test_vacuum(orc):
    sc = homogeneous_scene(scale=0.0, env=(0.2, 0.5, 1.0), radiance=(1.0, 1.0, 1.0), jitter=1, spp=4)
    L = orc.generate(sc, all_rays(48, 48))
    assert np.all(L == np.array([0.2, 0.5, 1.0]))


def test_degenerate_texels_are_zero(orc):
    sc = homogeneous_scene(env=(1.0, 1.0, 1.0), spp=4)
    L = orc.generate(sc, np.array([0, 49, 48 * 48 - 1]))
    assert np.all(L == 0.0)


def test_linearity(orc):
    sc = S.config(1, M=32, N=32, spp=8)
    ks = all_rays(32, 32)
    base = orc.generate(sc, ks)
    assert base.max() > 0
    two = orc.generate(dataclasses.replace(sc, light=dataclasses.replace(sc.light, radiance=(2.0, 2.0, 2.0))), ks)
    assert np.array_equal(two, 2 * base)
    env = (0.1, 0.2, 0.3)
    both = orc.generate(dataclasses.replace(sc, light=dataclasses.replace(sc.light, env=env)), ks)
    only_env = orc.generate(dataclasses.replace(sc, light=dataclasses.replace(sc.light, radiance=(0, 0, 0), env=env)), ks)
    assert np.allclose(both, base + only_env, rtol=1e-12, atol=1e-15)


def _gl(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def test_single_scatter_directional(orc):
    """max_bounces = 1: E[L] = rho f(d.w) E int sigma e^{-sigma (t - tn)} e^{-sigma s(t)} dt,
    s(t) the distance from x(t) to the box exit along the light direction."""
    rgb = (0.7, 0.5, 0.3)
    wl = np.array([0.3, 0.5, 0.81])
    wl /= np.linalg.norm(wl)
    lt = S.Light(kind=S.DIRECTIONAL, dir=tuple(wl))
    sc = homogeneous_scene(M=24, spp=4096, alpha=0.1, rgb=rgb, env=(0, 0, 0), radiance=(1.0, 1.0, 1.0),
                           max_bounces=1, g=0.3, light=lt)
    sigma = 1.0
    rng = np.random.default_rng(3)
    ks = S.random_rays(24, 24, 40, 9)
    L = orc.generate(sc, ks)
    zs = []
    for (o, d), Lk in zip(ray_geometry(orc, 24, 24, ks), L):
        ell, tn, tf = chord(o, d)
        fp = orc.lib().orc_hg_phase(0.3, float(d @ wl))
        if ell == 0:
            assert np.all(Lk == 0)
            continue
        ts, ws = _gl(64, tn, tf)
        integ = sum(w * sigma * math.exp(-sigma * (t - tn)) * math.exp(-sigma * chord(o + t * d, wl)[2])
                    for t, w in zip(ts, ws))
        mean = np.array(rgb) * fp * integ
        # each sample lies in [0, rho f E]: variance <= (rho f E)^2 / 4
        sd = np.array(rgb) * fp / 2 / math.sqrt(4096)
        zs.append((Lk - mean) / sd)
    zs = np.array(zs)
    assert np.abs(zs).max() < 5.5
    assert abs(zs.sum() / math.sqrt(zs.size)) < 5


def test_single_scatter_area_light(orc):
    """Area light, one scatter vertex: E[L] = rho int_t sigma e^{-sigma(t-tn)}
    int_A f(d.w) Le cos_l / r^2 e^{-sigma s} dA dt, with the light outside
    the box so the shadow segment ends at the box exit."""
    R = math.sqrt(3.0)
    lt = S.area_light(55, R)
    rgb = (0.6, 0.6, 0.6)
    sc = homogeneous_scene(M=16, spp=8192, alpha=0.1, rgb=rgb, env=(0, 0, 0), radiance=lt.radiance,
                           max_bounces=1, g=0.0, light=lt)
    ks = S.random_rays(16, 16, 12, 4)
    L = orc.generate(sc, ks)
    c0, e1, e2 = (np.array(v) for v in (lt.corner, lt.e1, lt.e2))
    nl = np.cross(e1, e2)
    area = np.linalg.norm(nl)
    nl /= area
    us, wu = _gl(12, 0.0, 1.0)
    for (o, d), Lk in zip(ray_geometry(orc, 16, 16, ks), L):
        ell, tn, tf = chord(o, d)
        if ell == 0:
            continue
        ts, wt = _gl(24, tn, tf)
        integ = 0.0
        for t, w in zip(ts, wt):
            x = o + t * d
            inner = 0.0
            for a, wa in zip(us, wu):
                for b, wb in zip(us, wu):
                    y = c0 + a * e1 + b * e2
                    v = y - x
                    r = np.linalg.norm(v)
                    om = v / r
                    cl = max(0.0, -nl @ om)
                    inner += wa * wb * (1 / (4 * math.pi)) * 4.0 * cl * area / r ** 2 * math.exp(-chord(x, om)[2])
            integ += w * math.exp(-(t - tn)) * inner
        mean = 0.6 * integ
        assert abs(Lk[0] - mean) < 6 * 0.6 * 4.0 * area / (4 * math.pi) / 4 / math.sqrt(8192) + 1e-3 * mean
