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


def slot_fields():
    a = [int(v) for v in re.search(r"kSlotA\[9\] = \{([^}]*)\}", SRC).group(1).split(",")]
    b = [int(v) for v in re.search(r"kSlotB\[9\] = \{([^}]*)\}", SRC).group(1).split(",")]
    return a, b


def test_slot_decode_gives_the_candidate_offsets():
    """slot t of a candidate set lies at a(t) F(k-1) + b(t) F(k) from its
    centre; a and b fit the 2- and 3-bit signed fields they are packed in"""
    a, b = slot_fields()
    assert len(a) == len(b) == 9
    assert all(-2 <= v <= 1 for v in a) and all(-4 <= v <= 3 for v in b)
    for k in range(2, 21):
        f1, f2, f3, f4 = fib(k - 1), fib(k), fib(k + 1), fib(k + 2)
        off = [0, f1, -f1, f2, -f2, f3, -f3, f4, -f4]
        assert [a[t] * f1 + b[t] * f2 for t in range(9)] == off, k


def test_slot_fields_round_trip_through_the_packing():
    """the packed constants, extracted as signed bit fields, give a and b back"""
    a, b = slot_fields()

    def pack(v, bits):
        return sum((x & ((1 << bits) - 1)) << (bits * t) for t, x in enumerate(v))

    def sbfe(word, off, bits):
        x = (word >> off) & ((1 << bits) - 1)
        return x - (1 << bits) if x >> (bits - 1) else x

    pa, pb = pack(a, 2), pack(b, 3)
    assert pa < 2 ** 31 and pb < 2 ** 31  # the device reads them as int
    assert [sbfe(pa, 2 * t, 2) for t in range(9)] == a
    assert [sbfe(pb, 3 * t, 3) for t in range(9)] == b


def test_slot_keys_order_like_distances():
    """32-bit keys (distance bits with the slot in the low four) order valid
    candidates by distance rounded down to 20 significant bits, ties by slot,
    and every invalid candidate (FLT_MAX) after every valid one"""
    inv = int(re.search(r"kInvalidKey = (0x[0-9a-f]+)u", SRC).group(1), 16)
    rng = np.random.default_rng(4)
    d2 = rng.uniform(0, 4, (20000, 9)).astype(np.float32)
    bits = d2.view(np.uint32)
    keys = (bits & ~np.uint32(15)) | np.arange(9, dtype=np.uint32)
    assert keys.max() < inv
    fmax = np.float32(np.finfo(np.float32).max).view(np.uint32)
    assert (fmax & ~np.uint32(15)) == inv
    order = np.argsort(keys, 1)
    trunc = (bits & ~np.uint32(15)).view(np.float32)
    srt = np.take_along_axis(trunc, order, 1)
    assert np.all(np.diff(srt, axis=1) >= 0)
    # rounding down loses at most 2^-19 of the value
    assert np.all((d2 - trunc) <= d2 * 2.0 ** -19)


def test_zone_constants():
    """the zone number's constants: 1 / log2(Phi^2) and pi sqrt(5)"""
    phi = (1 + 5 ** 0.5) / 2
    inv = float(re.search(r"kInvLog2Phi2 = ([0-9.]+)f;", SRC).group(1))
    assert abs(inv - np.log(2) / np.log(phi * phi)) < 1e-9
    ps5 = float(re.search(r"kPiSqrt5 = ([0-9.]+)f;", SRC).group(1))
    assert abs(ps5 - np.pi * np.sqrt(5)) < 1e-8
