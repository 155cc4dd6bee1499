"""Pins of the oracle's random numbers and scattering helpers.

Philox4x32-10 is compared with rocRAND's independent implementation (built
on the host from the ROCm headers); the phase function and its sampler with
textbook properties of the Henyey-Greenstein distribution; the tangent frame
with orthonormality."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    exe = str(tmp_path_factory.mktemp("philox") / "probe")
    src = os.path.join(HERE, "support", "philox_rocrand.cpp")
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_probe):
    rng = np.random.default_rng(11)
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [1, 2, 3, 4, 5, 6]]
    rows += rng.integers(0, 2 ** 32, (200, 6), dtype=np.uint64).tolist()
    # counters of the shape the path tracer uses: (ray, sample, bounce<<8|purpose, block)
    for k in (0, 65535, 2 ** 30 - 1):
        for s in (0, 7):
            for b in (0, 3):
                for p in range(4):
                    rows.append([k, s, (b << 8) | p, 1, 4001, 0])
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    got = np.array([orc.philox(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    assert np.array_equal(got, ref)


def test_uniform_conversion(orc):
    assert orc.uniform(0) == 0.0
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert orc.uniform(0x80000000) == 0.5
    # exact multiples of 2^-24, representable in binary32
    for x in (1 << 8, 12345 << 8, 0xDEADBEEF):
        u = orc.uniform(x)
        assert u * 2 ** 24 == int(u * 2 ** 24)
        assert float(np.float32(u)) == u


def test_philox_stream_uniformity(orc):
    """Chi-square over 64 bins of 40,000 uniforms from consecutive blocks."""
    u = []
    for b in range(10000):
        u.extend(orc.uniform(int(x)) for x in orc.philox([b, 3, (2 << 8) | 1, 0], [4001, 0]))
    u = np.array(u)
    h, _ = np.histogram(u, 64, (0, 1))
    e = len(u) / 64
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 120  # 63 dof: p ~ 1e-5
    # different purposes give uncorrelated streams
    a = np.array([orc.uniform(int(orc.philox([b, 0, 1, 0], [9, 0])[0])) for b in range(5000)])
    c = np.array([orc.uniform(int(orc.philox([b, 0, 3, 0], [9, 0])[0])) for b in range(5000)])
    assert abs(np.corrcoef(a, c)[0, 1]) < 0.05


@pytest.mark.parametrize("g", [0.0, 0.3, -0.5, 0.85])
def test_hg_phase_normalised(orc, g):
    # integral over the sphere: 2 pi int_{-1}^{1} f(mu) dmu = 1 (Gauss-Legendre)
    x, w = np.polynomial.legendre.leggauss(400)
    val = 2 * math.pi * sum(wi * orc.lib().orc_hg_phase(g, xi) for xi, wi in zip(x, w))
    assert abs(val - 1.0) < 1e-6


def test_hg_isotropic(orc):
    for mu in (-1.0, -0.3, 0.0, 0.7, 1.0):
        assert abs(orc.lib().orc_hg_phase(0.0, mu) - 1 / (4 * math.pi)) < 1e-15


@pytest.mark.parametrize("g", [0.0, 0.3, -0.5, 0.85])
def test_hg_sampler(orc, g):
    L = orc.lib()
    u = (np.arange(200000) + 0.5) / 200000  # stratified uniforms
    mu = np.array([L.orc_hg_sample_mu(g, x) for x in u])
    # the mean cosine of the HG distribution is g
    assert abs(mu.mean() - g) < 2e-4
    # the empirical CDF of the samples matches the integral of the phase
    # function's marginal 2 pi f(mu) (Gauss-Legendre on [-1, m])
    x, w = np.polynomial.legendre.leggauss(200)
    for m in np.linspace(-0.95, 0.95, 39):
        t = 0.5 * (m + 1) * x + 0.5 * (m - 1)
        cdf = 0.5 * (m + 1) * sum(wi * 2 * math.pi * L.orc_hg_phase(g, ti) for ti, wi in zip(t, w))
        assert abs((mu <= m).mean() - cdf) < 1e-4
    assert mu.min() >= -1 and mu.max() <= 1


def test_frame_orthonormal(orc):
    import ctypes as C
    rng = np.random.default_rng(4)
    ns = list(rng.standard_normal((500, 3))) + [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]),
                                                   np.array([1.0, 0, 0]), np.array([0, 1e-12, -1.0])]
    for n in ns:
        n = np.asarray(n, dtype=np.float64)
        n /= np.linalg.norm(n)
        t1 = np.zeros(3)
        t2 = np.zeros(3)
        orc.lib().orc_frame(n.ctypes.data_as(C.c_void_p), t1.ctypes.data_as(C.c_void_p),
                            t2.ctypes.data_as(C.c_void_p))
        B = np.stack([t1, t2, n])
        assert np.abs(B @ B.T - np.eye(3)).max() < 1e-14
        assert abs(np.linalg.det(B) - 1.0) < 1e-14
