"""Pins of the oracle's lookup (Sec. 2, image synthesis: front/back hit
points on S, nearest-neighbour query, 5x5 weighted texel fetches, nearest
sampling as the K = 1 case)."""
import math

import numpy as np
import pytest

import lfsynth as S


def line_camera(orc, M, N, i, j, W=33, H=17, back=2.0, R=math.sqrt(3.0)):
    """A camera on the line through R p_j -> R p_i, beyond p_i, looking along
    it: the centre pixel's ray enters S at R p_i and leaves at R p_j."""
    pi = orc.sf_points(M)[i]
    pj = orc.sf_points(N)[j]
    d = (pj - pi) / np.linalg.norm(pj - pi)
    eye = R * pi - back * R * d
    up = np.cross(d, [0.3, 0.2, 0.9])
    return S.Camera(eye=tuple(eye), target=tuple(eye + d), up=tuple(up / np.linalg.norm(up)), vfov=0.3)


@pytest.mark.parametrize("M,N", [(256, 256), (300, 128)])
def test_round_trip_nearest_sampling(orc, M, N):
    rng = np.random.default_rng(2)
    prm = S.Params(M=M, N=N)
    lf = rng.uniform(0, 1, M * N * 3).astype(np.float32)
    W, H = 33, 17
    for _ in range(40):
        i, j = int(rng.integers(M)), int(rng.integers(N))
        if M == N and i == j:
            continue
        cam = line_camera(orc, M, N, i, j, W, H)
        rgb, nn, _ = orc.lookup(lf, prm, [cam], W, H, 1, [[0, W // 2, H // 2]])
        assert nn[0].tolist() == [i, j]
        assert np.array_equal(rgb[0], lf[3 * (i * N + j): 3 * (i * N + j) + 3].astype(np.float64))


def test_constant_field_is_reproduced(orc):
    sc = S.config(1, M=256, N=256, views=2, width=40, height=30)
    lf = np.full(256 * 256 * 3, 0.37, np.float32)
    diag = 3 * (np.arange(256) * 257)
    for c in range(3):
        lf[diag + c] = 0.0  # degenerate texels i == j: weight 0, value irrelevant
    pix = orc.all_pixels(2, 40, 30)
    rgb, nn, _ = orc.lookup(lf, sc.params, sc.cams, 40, 30, 5, pix)
    hit = nn[:, 0] >= 0
    assert hit.sum() > 0.3 * len(pix) and (~hit).sum() > 0  # sphere covers part of the view
    assert np.abs(rgb[hit] - np.float32(0.37)).max() < 1e-15
    assert np.all(rgb[~hit] == 0.0) and np.all(nn[~hit] == -1)


def test_pixels_are_convex_combinations(orc):
    M = N = 128
    rng = np.random.default_rng(3)
    lf = rng.uniform(0, 1, M * N * 3).astype(np.float32)
    sc = S.config(1, M=M, N=N, views=1, width=24, height=24)
    pix = orc.all_pixels(1, 24, 24)
    rgb5, nn, _ = orc.lookup(lf, sc.params, sc.cams, 24, 24, 5, pix)
    rgb1, nn1, _ = orc.lookup(lf, sc.params, sc.cams, 24, 24, 1, pix)
    assert np.array_equal(nn, nn1)
    hit = nn[:, 0] >= 0
    assert np.all(rgb5[hit] >= 0) and np.all(rgb5[hit] <= 1)
    # blending differs from nearest sampling but stays near it on average
    assert np.abs(rgb5[hit] - rgb1[hit]).mean() < 0.35
    assert np.abs(rgb5[hit] - rgb1[hit]).max() > 1e-3


def test_adjoint_is_transpose(orc):
    M, N = 96, 80
    rng = np.random.default_rng(4)
    lf = rng.standard_normal(M * N * 3).astype(np.float32)
    sc = S.config(1, M=M, N=N, views=3, width=20, height=16)
    pix = orc.all_pixels(3, 20, 16)
    for K in (1, 5):
        img, _, _ = orc.lookup(lf, sc.params, sc.cams, 20, 16, K, pix)
        dimg = rng.standard_normal(img.shape)
        dlf = orc.lookup_adjoint(sc.params, sc.cams, 20, 16, K, pix, dimg)
        a = float((img * dimg).sum())
        b = float((lf.astype(np.float64) * dlf).sum())
        assert abs(a - b) < 1e-12 * (abs(a) + abs(b))


def test_view_margins_reported(orc):
    sc = S.config(1, M=256, N=256, views=1, width=32, height=32)
    lf = np.zeros(256 * 256 * 3, np.float32)
    _, nn, mg = orc.lookup(lf, sc.params, sc.cams, 32, 32, 5, orc.all_pixels(1, 32, 32))
    hit = nn[:, 0] >= 0
    assert np.all(mg[hit] > 0)
    assert np.all(mg[~hit][:, 1:] == 1e300)
