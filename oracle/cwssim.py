"""FP64 oracle of the complex-wavelet structural similarity (CW-SSIM) index.

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's quality report
call this module; the GPU library never does.

The paper reports CW-SSIM beside SSIM for its light-field views against
path-traced references (Sec. 3, image quality), naming only a
steerable pyramid of eight levels in total; this oracle reads that as eight
subbands (2 scales x 4 orientations).  The index is the one of Wang &
Simoncelli (2005) and Sampat et al. (2009): for
complex band-pass coefficients c_x, c_y of the same subband over a local
window,

    S = (2 |sum c_x conj(c_y)| + K) / (sum |c_x|^2 + sum |c_y|^2 + K),

averaged over window positions and subbands.  The subbands here are those
of a complex steerable filter bank defined in the DFT domain (a reading;
the paper does not give its transform):

* signed frequency of DFT index u of an n-point axis: f = u for 2u < n,
  u - n otherwise; angular frequency w = 2 pi f / n; r = |w|, theta =
  atan2(w_y, w_x);
* scale s = 0, 1 has the radial window R_s(r) = cos(pi/2 log2(r / r_s)) for
  |log2(r / r_s)| < 1, else 0, with r_s = pi / 2^(s+1) (one octave on each
  side of the centre; zero at r = 0, so a constant offset has no effect);
* orientation k = 0..3 has the one-sided angular window
  A_k(theta) = cos(d)^3 for |d| < pi/2, else 0, d = theta - pi k / 4
  wrapped to (-pi, pi] (one half-plane: the subband is analytic, complex);
* coefficients c = IDFT2(DFT2(x) R_s A_k), on the image's own periodic grid;
* windows: 7 x 7 uniform, at every position inside the image
  ((H - 6) x (W - 6));  K = 49 (0.01 data_range)^2, and a window whose
  numerator and denominator are both 0 counts as 1;
* the index of an RGB pair is the mean over the three channels, the 8
  subbands and the window positions.
"""
from __future__ import annotations

import numpy as np

SCALES = 2
ORIENTS = 4
WIN = 7


def signed_freq(n: int) -> np.ndarray:
    """Signed frequency f of each DFT index u of an n-point axis."""
    u = np.arange(n)
    return np.where(2 * u < n, u, u - n)


def band_filter(H: int, W: int, s: int, k: int) -> np.ndarray:
    """R_s(r) A_k(theta) on the H x W DFT grid ([v][u], FP64)."""
    wx = 2.0 * np.pi * signed_freq(W)[None, :] / W
    wy = 2.0 * np.pi * signed_freq(H)[:, None] / H
    r = np.hypot(wx, wy)
    theta = np.arctan2(wy, wx)
    rs = np.pi / 2.0 ** (s + 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        lr = np.log2(r / rs)
        radial = np.where(np.abs(lr) < 1.0, np.cos(0.5 * np.pi * lr), 0.0)
    d = theta - np.pi * k / ORIENTS
    d = np.angle(np.exp(1j * d))  # wrapped to (-pi, pi]
    angular = np.where(np.abs(d) < 0.5 * np.pi, np.cos(d) ** (ORIENTS - 1), 0.0)
    return radial * angular


def subband(x: np.ndarray, s: int, k: int) -> np.ndarray:
    """Complex coefficients of subband (s, k) of a 2-D image x [H][W]."""
    H, W = x.shape
    return np.fft.ifft2(np.fft.fft2(x.astype(np.float64)) * band_filter(H, W, s, k))


def window_sum(z: np.ndarray) -> np.ndarray:
    """Sum over every 7 x 7 window inside the array ([H-6][W-6])."""
    H, W = z.shape
    out = np.zeros((H - WIN + 1, W - WIN + 1), dtype=z.dtype)
    for dy in range(WIN):
        for dx in range(WIN):
            out += z[dy:dy + H - WIN + 1, dx:dx + W - WIN + 1]
    return out


def local_index(cx: np.ndarray, cy: np.ndarray, K: float) -> np.ndarray:
    """S at every window position of one subband."""
    num = 2.0 * np.abs(window_sum(cx * np.conj(cy))) + K
    den = window_sum(np.abs(cx) ** 2) + window_sum(np.abs(cy) ** 2) + K
    return np.where(den > 0.0, num / np.where(den > 0.0, den, 1.0), 1.0)


def cw_ssim(a, b, data_range: float = 1.0) -> np.ndarray:
    """Mean CW-SSIM [n] of image pairs [n, H, W, 3]."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    K = WIN * WIN * (0.01 * data_range) ** 2
    out = []
    for x, y in zip(a, b):
        vals = []
        for c in range(x.shape[-1]):
            for s in range(SCALES):
                for k in range(ORIENTS):
                    vals.append(local_index(subband(x[..., c], s, k), subband(y[..., c], s, k), K).mean())
        out.append(float(np.mean(vals)))
    return np.array(out)
