"""Pin of the direction a path takes after a real collision (the scatter step
of the path tracer that Sec. 2 relies on, read volumetrically).

Set-up: homogeneous medium of extinction sigma and albedo 1, no light, a
constant environment of radiance 1, two scatter vertices and no origin
jitter.  A sample then returns exactly 1 when the path leaves the box before
its second real collision, and 0 otherwise (the second vertex is the last
one and adds nothing without a light).  Its expectation for the ray o + t d
with chord [tn, tf] is

    E = e^{-sigma (tf - tn)}
        + int_tn^tf sigma e^{-sigma (t - tn)}
              int_{S^2} p_g(d . w) e^{-sigma l(o + t d, w)} dw dt,

with p_g the Henyey-Greenstein density of the cosine between the old and
the new direction and l(x, w) the distance from x to the box exit along w.
The inner integral is taken over (mu, phi) with w = mu d + sqrt(1 - mu^2)
(cos phi a + sin phi b) for any orthonormal (a, b) completing d: Gauss-
Legendre in t and mu, the trapezoid rule in phi.

The expectation depends on the direction distribution: a collision near the
entry face escapes easily backwards and rarely forwards, so g = +0.6 and
g = -0.6 give clearly different answers (checked below, so that the test
keeps its power).  A sign error in mu (back- instead of forward scattering),
a wrong azimuth or a direction that is not unit length moves the oracle away
from the quadrature."""
import math

import numpy as np
import pytest

import lfsynth as S

SIGMA = 1.5      # extinction per world unit: scale 10 x alpha 0.15
SPP = 1 << 16
M = 16


def scene(g):
    vol = S.constant_volume(8, 1.0)
    med = S.Medium(S.constant_lut((1.0, 1.0, 1.0), SIGMA / 10.0), 10.0)
    lt = S.Light(kind=S.DIRECTIONAL, dir=(0.0, 0.0, 1.0), radiance=(0.0, 0.0, 0.0), env=(1.0, 1.0, 1.0))
    prm = S.Params(M=M, N=M, spp=SPP, max_bounces=2, g=g, seed=2024, jitter=0)
    return S.Scene("scatter-direction", vol, med, lt, prm)


def exit_distance(X, W, lo=-1.0, hi=1.0):
    """Distance from points X (inside the box) to the box exit along W.
    X: [..., 3], W: [..., 3] (broadcast)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t_hi = (hi - X) / W
        t_lo = (lo - X) / W
    t = np.where(W > 0, t_hi, np.where(W < 0, t_lo, np.inf))
    return np.maximum(t.min(-1), 0.0)


def chord(o, d, lo=-1.0, hi=1.0):
    t0, t1 = 0.0, math.inf
    for a in range(3):
        if d[a] == 0:
            continue
        ta, tb = (lo - o[a]) / d[a], (hi - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return (t0, t1) if t1 > t0 else (0.0, 0.0)


def hg_density(g, mu):
    """Henyey-Greenstein density over the sphere (integrates to 1 over dw)."""
    return (1.0 - g * g) / (4.0 * math.pi * (1.0 + g * g - 2.0 * g * mu) ** 1.5)


def escape_probability(o, d, g, nt=48, nmu=96, nphi=192, attenuate=True):
    """E above by quadrature; attenuate=False replaces e^{-sigma l} by 1 (then
    E = 1: the first-collision density and p_g are normalised)."""
    tn, tf = chord(o, d)
    if tf <= tn:
        return 1.0
    # any orthonormal completion of d (the integral does not depend on it)
    helper = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    a = np.cross(d, helper)
    a /= np.linalg.norm(a)
    b = np.cross(d, a)
    xt, wt = np.polynomial.legendre.leggauss(nt)
    t = 0.5 * (tf - tn) * xt + 0.5 * (tf + tn)
    wt = 0.5 * (tf - tn) * wt
    xm, wm = np.polynomial.legendre.leggauss(nmu)
    phi = 2.0 * math.pi * np.arange(nphi) / nphi
    st = np.sqrt(1.0 - xm * xm)
    Wd = (xm[:, None, None] * d + st[:, None, None] *
          (np.cos(phi)[None, :, None] * a + np.sin(phi)[None, :, None] * b))      # [nmu][nphi][3]
    X = o + t[:, None] * d                                                         # [nt][3]
    ell = exit_distance(X[:, None, None, :], Wd[None])                             # [nt][nmu][nphi]
    esc = np.exp(-SIGMA * ell) if attenuate else np.ones_like(ell)
    inner = (esc.mean(-1) * 2.0 * math.pi * hg_density(g, xm) * wm).sum(-1)
    first = SIGMA * np.exp(-SIGMA * (t - tn))
    return math.exp(-SIGMA * (tf - tn)) + float((wt * first * inner).sum())


def test_quadrature_self_checks():
    """The quadrature itself: p_g integrates to 1 over the sphere and has mean
    cosine g (the defining property of the Henyey-Greenstein g, g > 0
    forward); without the second attenuation E is exactly 1; the exit
    distances agree with a scalar slab clip at random interior points; and
    the isotropic inner integral at the box centre equals a fine direct
    average of e^{-sigma l} over a Fibonacci sphere."""
    xm, wm = np.polynomial.legendre.leggauss(96)
    for g in (0.6, -0.6, 0.0, 0.3):
        assert abs((2 * math.pi * hg_density(g, xm) * wm).sum() - 1.0) < 1e-10
        assert abs((2 * math.pi * xm * hg_density(g, xm) * wm).sum() - g) < 1e-10
    o = np.array([-1.7, 0.05, 0.1])
    d = np.array([1.0, 0.3, -0.2])
    d /= np.linalg.norm(d)
    assert abs(escape_probability(o, d, 0.6, attenuate=False) - 1.0) < 1e-12
    rng = np.random.default_rng(5)
    X = rng.uniform(-0.9, 0.9, (200, 3))
    Wr = rng.standard_normal((200, 3))
    Wr /= np.linalg.norm(Wr, axis=1, keepdims=True)
    got = exit_distance(X, Wr)
    ref = np.array([chord(x, w)[1] for x, w in zip(X, Wr)])
    assert np.abs(got - ref).max() < 1e-12
    n = 200000
    i = np.arange(n)
    z = 1 - (2 * i + 1) / n
    ph = 2 * math.pi * ((i * (math.sqrt(5) - 1) / 2) % 1.0)
    Wf = np.stack([np.sqrt(1 - z * z) * np.cos(ph), np.sqrt(1 - z * z) * np.sin(ph), z], 1)
    direct = np.exp(-SIGMA * exit_distance(np.zeros(3), Wf)).mean()
    phi = 2 * math.pi * np.arange(192) / 192
    st = np.sqrt(1 - xm * xm)
    Wd = np.stack([st[:, None] * np.cos(phi), st[:, None] * np.sin(phi), np.broadcast_to(xm[:, None], (96, 192))], -1)
    quad = (np.exp(-SIGMA * exit_distance(np.zeros(3), Wd)).mean(-1) * 0.5 * wm).sum()
    assert abs(quad - direct) < 1e-3


@pytest.mark.parametrize("g", [0.6, -0.6, 0.0])
def test_scatter_direction_two_vertices(orc, g):
    # rays whose chord through the box is 2.0-2.8 (the first collision then
    # falls well inside, where the scattered direction decides the escape)
    ks = np.array([60, 43, 149, 200, 241, 72, 84])
    Po = orc.sf_points(M)
    R = math.sqrt(3.0)
    L = orc.generate(scene(g), ks)
    assert np.all(L[:, 0] == L[:, 1]) and np.all(L[:, 0] == L[:, 2])
    zs = []
    for k, Lk in zip(ks, L[:, 0]):
        i, j = divmod(int(k), M)
        o = R * Po[i]
        d = Po[j] - Po[i]
        d /= np.linalg.norm(d)
        p = escape_probability(o, d, g)
        sd = math.sqrt(p * (1 - p) / SPP)
        # the estimator has power: the mirrored phase function is far away
        if g != 0.0:
            assert abs(escape_probability(o, d, -g) - p) > 50 * sd
        zs.append((Lk - p) / sd)
    zs = np.array(zs)
    # each sample is a Bernoulli variable; 1e-3 allows for the quadrature
    assert np.all(np.abs(zs) < 5.0), zs
    assert abs(zs.sum() / math.sqrt(len(zs))) < 5.0
