"""Pins of the oracle's CW-SSIM (complex-wavelet SSIM, Wang & Simoncelli 2005,
Sampat et al. 2009), the second index the paper reports for its views
against path-traced references (Sec. 3, image quality)."""
import numpy as np
import pytest

from oracle import cwssim as cw


def test_angular_windows_form_a_steerable_basis():
    """cos^3 windows at 4 orientations: the energy of direction theta and of
    its opposite add to 4 C(6,3) / 2^6 = 1.25 for every theta (the identity
    sum_k cos^6(theta - pi k / 4) = 5/4)."""
    H = W = 64
    tot = sum(cw.band_filter(H, W, 0, k) ** 2 for k in range(cw.ORIENTS))
    # pair (u, v) with (-u, -v) on the grid (both inside the Nyquist range)
    fu, fv = cw.signed_freq(W), cw.signed_freq(H)
    for v in range(H):
        for u in range(W):
            if 2 * abs(fu[u]) >= W or 2 * abs(fv[v]) >= H:
                continue
            r = np.hypot(2 * np.pi * fu[u] / W, 2 * np.pi * fv[v] / H)
            lr = np.log2(r / (np.pi / 2)) if r > 0 else -np.inf
            if not abs(lr) < 1:
                continue
            R2 = np.cos(0.5 * np.pi * lr) ** 2
            opp = tot[(-v) % H, (-u) % W]
            assert abs((tot[v, u] + opp) / R2 - 1.25) < 1e-12, (u, v)


def test_radial_windows_split_the_octave():
    """Along theta = 0 (where A_0 = 1): R_0^2 + R_1^2 = 1 between the two
    centres (pi/4 <= r <= pi/2); every filter is 0 at DC."""
    H = W = 96
    r = 2 * np.pi * cw.signed_freq(W) / W
    f0 = cw.band_filter(H, W, 0, 0)[0] ** 2 + cw.band_filter(H, W, 1, 0)[0] ** 2
    sel = (r >= np.pi / 4) & (r <= np.pi / 2)
    assert sel.sum() > 5
    np.testing.assert_allclose(f0[sel], 1.0, atol=1e-12)
    for s in range(cw.SCALES):
        for k in range(cw.ORIENTS):
            assert cw.band_filter(H, W, s, k)[0, 0] == 0.0


def test_subband_equals_explicit_dft():
    """The FFT route against DFT matrices written from the definition
    (X = E_H x E_W^T, c = conj(E_H) (X F) conj(E_W)^T / (H W)), on an odd
    and an even axis."""
    H, W = 9, 12
    rng = np.random.default_rng(3)
    x = rng.normal(size=(H, W))
    EH = np.exp(-2j * np.pi * np.outer(np.arange(H), np.arange(H)) / H)
    EW = np.exp(-2j * np.pi * np.outer(np.arange(W), np.arange(W)) / W)
    X = EH @ x @ EW.T
    for s in range(cw.SCALES):
        for k in range(cw.ORIENTS):
            F = cw.band_filter(H, W, s, k)
            ref = np.conj(EH) @ (X * F) @ np.conj(EW).T / (H * W)
            np.testing.assert_allclose(cw.subband(x, s, k), ref, atol=1e-12)


def test_window_sum_brute_force():
    rng = np.random.default_rng(4)
    z = rng.normal(size=(11, 13))
    got = cw.window_sum(z)
    assert got.shape == (5, 7)
    for y in range(5):
        for x in range(7):
            assert abs(got[y, x] - z[y:y + 7, x:x + 7].sum()) < 1e-12


@pytest.fixture(scope="module")
def imgs():
    rng = np.random.default_rng(1)
    a = rng.uniform(0, 1, (2, 30, 41, 3))
    b = np.clip(a + rng.normal(0, 0.2, a.shape), 0, 1)
    return a, b


def test_identity_offset_and_sign(imgs):
    a, _ = imgs
    np.testing.assert_allclose(cw.cw_ssim(a, a), 1.0, atol=1e-12)
    # the band-pass filters are 0 at DC: a constant offset changes nothing
    np.testing.assert_allclose(cw.cw_ssim(a, a + 0.37), 1.0, atol=1e-12)
    # |sum c conj(-c)| = sum |c|^2: a sign flip changes nothing (K = 0)
    np.testing.assert_allclose(cw.cw_ssim(a, -a, data_range=0.0), 1.0, atol=1e-12)


@pytest.mark.parametrize("s", [0.5, 2.0, 3.0])
def test_scaled_image_closed_form(imgs, s):
    """c_y = s c_x gives 2 s / (1 + s^2) in every window (K = 0)."""
    a, _ = imgs
    np.testing.assert_allclose(cw.cw_ssim(a, s * a, data_range=0.0), 2 * s / (1 + s * s), atol=1e-12)


def test_symmetry_range_and_zero_images(imgs):
    a, b = imgs
    ab, ba = cw.cw_ssim(a, b), cw.cw_ssim(b, a)
    np.testing.assert_allclose(ab, ba, atol=1e-14)
    assert np.all((ab > 0.0) & (ab < 1.0))
    z = np.zeros((1, 10, 10, 3))
    np.testing.assert_allclose(cw.cw_ssim(z, z, data_range=0.0), 1.0)
    # noise is far less similar than a noisy copy
    rng = np.random.default_rng(9)
    assert cw.cw_ssim(a[:1], rng.uniform(0, 1, a[:1].shape))[0] < ab[0]


def test_local_index_is_phase_sensitive():
    """|sum c_x conj(c_y)|, not sum |c_x conj(c_y)|: c_x = 1 and c_y = +1 on
    25 cells, -1 on 24 cells of one 7 x 7 window give (2 * 1) / (49 + 49)."""
    cx = np.ones((7, 7), complex)
    cy = np.ones(49, complex)
    cy[25:] = -1.0
    cy = cy.reshape(7, 7)
    got = cw.local_index(cx, cy, 0.0)
    assert got.shape == (1, 1)
    assert abs(got[0, 0] - 2.0 / 98.0) < 1e-15
    # a common phase rotation of c_y is invisible
    assert abs(cw.local_index(cx, 1j * cx, 0.0)[0, 0] - 1.0) < 1e-15
