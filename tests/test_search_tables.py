"""Host checks of two constant tables of the lookup's nearest-point search
(inverse spherical-Fibonacci mapping, Sec. 2), read from the device header:

- the azimuth polynomial that places a query in a lattice cell must stay
  within a few 1e-7 rad of atan2 over all octants;
- the slot tables that let the first candidate set reuse the four lattice
  corners' distances must name, for each nearest corner, exactly the slots
  whose index offsets reach the other three corners (corner s at offset
  (s & 1) F(k) + (s >> 1) F(k+1) from corner 0), and the other five slots.
"""
import os
import re

import numpy as np

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1903_03837_amd", "csrc", "sf_search.hpp")
SRC = open(HDR).read()


def fib(k):
    a, b = 0, 1
    for _ in range(k):
        a, b = b, a + b
    return a


def azimuth_coeffs():
    body = re.search(r"float sf_azimuth\(float y, float x\) \{(.*?)\n\}", SRC, re.S).group(1)
    first = float(re.search(r"float p = (-?[0-9.e+-]+)f;", body).group(1))
    rest = [float(c) for c in re.findall(r"p = fmaf\(p, s, (-?[0-9.e+-]+)f\);", body)]
    assert len(rest) == 7
    return [first] + rest


def azimuth(y, x):
    """the device formula in FP32 (each fmaf rounded once through FP64)"""
    f = np.float32
    c = [f(v) for v in azimuth_coeffs()]
    ax, ay = np.abs(x).astype(f), np.abs(y).astype(f)
    mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(mx > 0, (mn / mx).astype(f), f(0))
    s = (t * t).astype(f)
    p = np.full_like(t, c[0])
    for ci in c[1:]:
        p = (p.astype(np.float64) * s + ci).astype(f)
    r = (t * p).astype(f)
    r = np.where(ay > ax, (f(np.pi / 2) - r).astype(f), r)
    r = np.where(x < 0, (f(np.pi) - r).astype(f), r)
    return np.copysign(r, y).astype(f)


def test_azimuth_polynomial_within_a_few_1e7_rad():
    rng = np.random.default_rng(11)
    ang = np.concatenate([rng.uniform(-np.pi, np.pi, 400000),
                          np.arange(-8, 9) * (np.pi / 4)])  # axes and octant edges
    rad = rng.uniform(0.05, 1.0, ang.size)
    x = (rad * np.cos(ang)).astype(np.float32)
    y = (rad * np.sin(ang)).astype(np.float32)
    got = azimuth(y, x).astype(np.float64)
    ref = np.arctan2(y.astype(np.float64), x.astype(np.float64))
    err = np.abs(got - ref)
    err = np.minimum(err, 2 * np.pi - err)  # +-pi on the seam are the same azimuth
    assert err.max() < 5e-7, err.max()


def test_azimuth_on_the_axes():
    one, zero = np.float32(1), np.float32(0)
    assert azimuth(np.array([zero]), np.array([one]))[0] == 0
    assert abs(azimuth(np.array([one]), np.array([zero]))[0] - np.pi / 2) < 2e-7
    assert abs(azimuth(np.array([-one]), np.array([zero]))[0] + np.pi / 2) < 2e-7
    assert abs(abs(azimuth(np.array([zero]), np.array([-one]))[0]) - np.pi) < 2e-7


def slot_tables():
    corner = re.search(r"kCornerSlot\[4\]\[4\] = \{(.*?)\};", SRC, re.S).group(1)
    opens = re.search(r"kOpenSlot\[4\]\[5\] = \{(.*?)\};", SRC, re.S).group(1)
    rows = lambda s: [[int(v) for v in r.split(",")] for r in re.findall(r"\{([^{}]*)\}", s)]
    return rows(corner), rows(opens)


def test_corner_slots_reach_the_other_corners():
    corner, opens = slot_tables()
    assert len(corner) == 4 and len(opens) == 4
    for k in range(3, 21):
        f1, f2, f3, f4 = fib(k - 1), fib(k), fib(k + 1), fib(k + 2)
        off = [0, f1, -f1, f2, -f2, f3, -f3, f4, -f4]  # the candidate slots' offsets
        pos = lambda s: (s & 1) * f2 + (s >> 1) * f3
        for s in range(4):
            for s2 in range(4):
                assert off[corner[s][s2]] == pos(s2) - pos(s), (k, s, s2)
            assert sorted(corner[s] + opens[s]) == list(range(9)), s
