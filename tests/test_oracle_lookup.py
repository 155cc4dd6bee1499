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


def test_upper_hemisphere_is_first_half(orc):
    """z_i falls with i, so the origins with z > 0 are the first floor(M/2)
    indices (Sec. 3 stores that half of P_o)."""
    for M in (12288, 301, 2):
        z = orc.sf_points(M)[:, 2]
        assert np.all(np.diff(z) < 0)
        assert np.all(z[: M // 2] > 0) and np.all(z[(M + 1) // 2:] < 0)


@pytest.mark.parametrize("M,N", [(300, 128), (256, 256)])
def test_stored_origin_rows_renormalise(orc, M, N):
    """Lookup over the stored rows i < rows is the full-M lookup restricted to
    those origins and renormalised: with ind(i) = [i < rows],
    half(g) = full(g * ind) / full(ind) wherever full(ind) > 0, else 0."""
    rows = M // 2
    V, W, H = 3, 36, 28
    rng = np.random.default_rng(11)
    cams = S.seam_cameras(math.sqrt(3.0))
    half = S.Params(M=M, N=N, origin_rows=rows)
    full = S.Params(M=M, N=N)
    pix = orc.all_pixels(V, W, H)
    g = rng.uniform(0.1, 1.0, (M, N, 3)).astype(np.float32)
    ind = np.zeros((M, N, 3), np.float32)
    ind[:rows] = 1.0
    gi = (g * ind).astype(np.float32)
    for K in (1, 5, 9):
        h, nn_h, _ = orc.lookup(g[:rows], half, cams, W, H, K, pix)
        f_gi, nn_f, _ = orc.lookup(gi, full, cams, W, H, K, pix)
        f_ind, _, _ = orc.lookup(ind, full, cams, W, H, K, pix)
        assert np.array_equal(nn_h, nn_f)
        cov = f_ind[:, 0] > 0
        hit = nn_f[:, 0] >= 0
        # the views see both hemispheres and, for K > 1, the seam between them
        assert (hit & cov).sum() > 0.1 * hit.sum() and (hit & ~cov).sum() > 0.1 * hit.sum()
        if K > 1:
            assert ((f_ind[:, 0] > 0) & (f_ind[:, 0] < 1 - 1e-9)).sum() > 0
        else:
            assert np.array_equal(cov, hit & (nn_f[:, 0] < rows))
        ref = f_gi[cov] / f_ind[cov]
        assert np.abs(h[cov] - ref).max() <= 1e-12
        assert np.all(h[~cov] == 0.0)


def test_stored_origin_rows_adjoint_is_transpose(orc):
    M, N, rows = 96, 80, 48
    rng = np.random.default_rng(12)
    cams = S.seam_cameras(math.sqrt(3.0))
    prm = S.Params(M=M, N=N, origin_rows=rows)
    lf = rng.standard_normal(rows * N * 3).astype(np.float32)
    pix = orc.all_pixels(3, 20, 16)
    for K in (1, 5):
        img, _, _ = orc.lookup(lf, prm, cams, 20, 16, K, pix)
        dimg = rng.standard_normal(img.shape)
        dlf = orc.lookup_adjoint(prm, cams, 20, 16, K, pix, dimg)
        assert dlf.shape == (rows * N * 3,)
        a = float((img * dimg).sum())
        b = float((lf.astype(np.float64) * dlf).sum())
        assert abs(a - b) < 1e-12 * (abs(a) + abs(b))
