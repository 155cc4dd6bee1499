"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Bars:
  - point coordinates: within 4e-7 of the FP64 values (FP32 rounding);
  - indices (nearest point, neighbour sets): bit-exact wherever the oracle's
    decision margin exceeds the FP32 band; inside the band the GPU's choice
    must be one of the near-tied candidates;
  - radiance: aggregate relative L1 error <= 1e-3 with the same random stream;
  - lookup RGB on decided pixels: the FP32 view ray moves a hit point by
    ~2.5e-7 R, which shifts a tent weight by ~1e-6 / r (r = sqrt(4 pi / n),
    the unit-sphere filter radius); over a field of value range D the pixel
    moves by at most LOOKUP_C / r * D (measured 1.2e-5 / r * D on random
    fields, which have the largest texel-to-texel jumps).
Inputs are seeded synthetic scenes (lfsynth) or seeded random light fields,
never outputs of the GPU path.
"""
import dataclasses
import math
import os

import numpy as np
import pytest
import torch

import lfsynth as S
import radiance_bars as bars

pytestmark = pytest.mark.gpu

RAD_TOL = 1e-3
# FP32 band of the nearest / K-th decisions, relative to the area per point
BAND = 1e-4
LOOKUP_C = 3e-5
# bounds on the share of flipped values (see radiance_bars), a few times the
# rate measured on MI355X for each workload (c1: 0 of 195840 values; c2 and c5:
# 3 of 60000)
FLIPS = {"c1": 1e-4, "c2": 3e-4, "c5": 3e-4}


def lookup_tol(M, N, lf):
    # a tent weight moves by ~1e-6 / r under the FP32 rounding of the hits,
    # most for the finer of the two point sets (the larger n)
    r = math.sqrt(4 * math.pi / max(M, N))
    return LOOKUP_C / r * float(lf.max() - lf.min())


def check_pixels(g_img, rgb, tol):
    err = np.abs(g_img - rgb)
    assert err.max() <= tol, (err.max(), tol)
    assert np.quantile(err, 0.99) <= tol / 10


@pytest.fixture(scope="module")
def lp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1903_03837_amd as lp
    lp.library()
    return lp


def rel_l1(got, ref):
    return float(np.abs(got - ref).sum() / np.abs(ref).sum())


def nondegenerate(M, N, ks):
    ks = np.asarray(ks)
    return ks[~((M == N) & ((ks // N) == (ks % N)))]


def gpu_field(lp, sc, dtype="f32", sample=None, stats=False):
    vol, med, light, prm, _ = lp.device_scene(sc)
    st = torch.zeros(5, dtype=torch.int64, device="cuda") if stats else None
    smp = None
    if sample is not None:
        smp = lp.Medium(torch.from_numpy(sample.lut).cuda(), sample.scale)
    lf = lp.generate(vol, med, light, prm, dtype=dtype, sample=smp, stats=st)
    torch.cuda.synchronize()
    out = lf.float().reshape(-1, 3).cpu().numpy().astype(np.float64)
    return (out, st.cpu().numpy()) if stats else out


# ------------------------------------------------------------------ SF points
@pytest.mark.parametrize("n", [1, 2, 5, 256, 2048, 32768, 65535])
def test_points(lp, orc, n):
    xyz, _, _ = lp.points(n)
    torch.cuda.synchronize()
    got = xyz.cpu().numpy().astype(np.float64)
    ref = orc.sf_points(n)
    assert np.abs(got - ref).max() < 4e-7


def unit_queries(n_rand, seed, extra=()):
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((n_rand, 3))
    q = np.concatenate([q, np.array([[0, 0, 1.0], [0, 0, -1.0], [-1.0, 1e-7, 0.0], [-1.0, -1e-7, 0.3]])] +
                       [np.asarray(e) for e in extra])
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


@pytest.mark.parametrize("n,K", [(16, 5), (256, 5), (2048, 5), (8192, 5), (32768, 5), (2048, 1), (32768, 1),
                                 (2048, 9), (32768, 9), (65535, 3)])
def test_neighbor_query(lp, orc, n, K):
    P = orc.sf_points(n)
    rng = np.random.default_rng(n)
    # every point itself, points jittered by 0.3 spacings, random queries, poles, seam
    pts = P[rng.choice(n, min(n, 2000), replace=False)]
    jit = pts + 0.3 * math.sqrt(4 * math.pi / n) * rng.standard_normal(pts.shape)
    q = unit_queries(6000, n + 1, extra=(pts, jit))
    _, idx, w = lp.points(n, torch.from_numpy(q).cuda(), K, want_xyz=False)
    torch.cuda.synchronize()
    g_idx = idx.cpu().numpy()
    g_w = w.cpu().numpy()
    o_idx, o_w, o_d2, mg, cnt = orc.neighbors_batch(n, q.astype(np.float64), K)
    area = 4 * math.pi / n
    clear = (mg[:, 0] / area > BAND) & (mg[:, 1] > 1e-3) & (mg[:, 2] / area > BAND)
    assert clear.mean() > 0.99
    # the nearest point and the K-set are unique outside the bands; the order
    # of near-equidistant members inside the set is not (lattice neighbours
    # at i +- F sit at almost equal distances), so it must only be sorted by
    # the oracle's distances to within the band
    assert np.array_equal(g_idx[clear, 0], o_idx[clear, 0])
    assert np.array_equal(np.sort(g_idx[clear], 1), np.sort(o_idx[clear], 1))
    qc = q[clear].astype(np.float64)
    gi = g_idx[clear]
    d2g = np.sum((P[np.clip(gi, 0, n - 1)] - qc[:, None, :]) ** 2, -1)
    d2g[gi < 0] = 1e30  # missing entries last (finite: two of them in a row differ by 0, not NaN)
    assert np.all(np.diff(d2g, axis=1) >= -BAND * area)
    og = np.argsort(g_idx[clear], 1)
    oo = np.argsort(o_idx[clear], 1)
    assert np.abs(np.take_along_axis(g_w[clear], og, 1) - np.take_along_axis(o_w[clear], oo, 1)).max() < 1e-4
    # near-tied nearest: the GPU's pick is within the band of the best
    amb = ~clear
    if amb.any():
        Pq = P[np.clip(g_idx[amb, 0], 0, n - 1)]
        d_gpu = np.sum((Pq - q[amb].astype(np.float64)) ** 2, 1)
        assert np.all(d_gpu - o_d2[amb, 0] <= BAND * area)


# ------------------------------------------------------------------ generation
def test_generate_c1_full(lp, orc):
    """Tiny blob workload at full size: all 65,536 rays against the oracle."""
    sc = S.config(1)
    got, st = gpu_field(lp, sc, stats=True)
    ks = np.arange(256 * 256)
    ref, ost = orc.generate(sc, ks, stats=True)
    assert np.all(got[ks[(ks // 256) == (ks % 256)]] == 0.0)
    nd = nondegenerate(256, 256, ks)
    print(f"c1: collisions/sample GPU {st[0] / st[3]:.3f} oracle {ost[0] / ost[3]:.3f}")
    bars.check(got[nd], ref[nd], FLIPS["c1"], "c1 (all rays)")
    assert st[3] == ost[3]
    assert abs(st[0] / ost[0] - 1) < 1e-3 and abs(st[1] / ost[1] - 1) < 1e-3


def test_waves_per_simd_leaves_results_unchanged(lp):
    """The forward tracer budgeted for 3 or 4 waves per SIMD runs the same
    code on the same random numbers: the light field (plain, with work
    counts, with frozen sampling), the kept sample radiance and the
    ground-truth views are bit-identical; other values are rejected."""
    sc = S.config(2, M=256, N=256, spp=8, views=2, width=96, height=64)
    vol, med, light, prm, cams = lp.device_scene(sc)
    out = {}
    for w in (3, 4):
        p = dataclasses.replace(prm, waves_per_simd=w)
        srad = torch.zeros((256, 256, 8, 3), dtype=torch.float32, device="cuda")
        stats = torch.zeros(5, dtype=torch.int64, device="cuda")
        lf = lp.generate(vol, med, light, p, stats=stats, sample_radiance=srad)
        frozen = lp.generate(vol, lp.Medium(med.lut * 0.9, med.scale), light, p, sample=med)
        views = lp.render_views(vol, med, light, p, cams, 96, 64)
        torch.cuda.synchronize()
        out[w] = (lf, srad, stats, frozen, views)
    for a, b in zip(out[3], out[4]):
        assert torch.equal(a, b)
    with pytest.raises(lp.LumiPathError):
        lp.generate(vol, med, light, dataclasses.replace(prm, waves_per_simd=5))


def test_generate_c5_sampled(lp, orc):
    """Differentiation workload (f32 volume) at full size, 20000 sampled rays."""
    sc = S.config(5)
    got = gpu_field(lp, sc)
    ks = S.random_rays(1024, 1024, 20000, 55)
    ref = orc.generate(sc, ks)
    bars.check(got[ks], ref, FLIPS["c5"], "c5 (20000 rays)")


def test_generate_c2_full_size_sampled(lp, orc):
    """CT-like workload at full size (4.19M rays, 64 spp, 8 bounces, area
    light), in the configuration the benchmark times; 20000 sampled rays."""
    sc = S.config(2)
    got = gpu_field(lp, sc)
    ks = S.random_rays(2048, 2048, 20000, 22)
    ref = orc.generate(sc, ks)
    bars.check(got[ks], ref, FLIPS["c2"], "c2 (20000 rays)")
    assert np.all(np.isfinite(got))


def test_generate_ragged_and_tiny(lp, orc):
    """Sizes that are not multiples of the 8 x 8 tile, M != N, M = N = 1."""
    for M, N in [(13, 7), (1, 1), (3, 40), (37, 37)]:
        sc = S.config(1, M=M, N=N, spp=4)
        got = gpu_field(lp, sc)
        ks = np.arange(M * N)
        ref = orc.generate(sc, ks)
        nd = nondegenerate(M, N, ks)
        if M == N:
            assert np.all(got[ks[(ks // N) == (ks % N)]] == 0.0)
        if len(nd) and np.abs(ref[nd]).sum() > 0:
            assert rel_l1(got[nd], ref[nd]) <= RAD_TOL, (M, N)


@pytest.mark.parametrize("M,N", [(65535, 8), (8, 65535)])
def test_generate_largest_point_sets(lp, orc, M, N):
    """The largest SF sets generation takes (65535 points: the FP64 golden-
    ratio step at its largest index) as origins or as directions, with a
    tiny other set (524 280 rays, 4 spp): 20000 sampled rays against the
    oracle, and every texel finite."""
    sc = S.config(1, M=M, N=N, spp=4)
    got = gpu_field(lp, sc)
    ks = S.random_rays(M, N, 20000, 73)
    ref = orc.generate(sc, ks)
    assert np.all(np.isfinite(got))
    bars.check(got[ks], ref, FLIPS["c1"] * 5, f"M={M} N={N} (20000 rays)")


# ------------------------------------------------------------ majorant grid
@pytest.mark.parametrize("c,G,vol_n", [(1, 16, None), (1, 7, None), (2, 16, 64), (3, 16, 64), (5, 11, 32)])
def test_majorant_grid_matches_oracle(lp, orc, c, G, vol_n):
    """Cell majorants: the oracle's FP64 values rounded once to FP32 (u8
    linear, u16 linear, u16 in 8^3 bricks, f32; G dividing n or not)."""
    sc = S.config(c, vol_n=vol_n) if vol_n else S.config(c)
    sc = sc.with_params(grid=G)
    vol, med, _, prm, _ = lp.device_scene(sc)
    got = lp.majorant_grid(vol, med, prm).cpu().numpy()
    ref = orc.majorant_grid(sc.volume, sc.medium, sc.params).astype(np.float32)
    assert np.array_equal(got, ref)


def test_generate_global_majorant(lp, orc):
    """grid = 0 tracks against the one global majorant."""
    sc = S.config(1, M=96, N=96, spp=8, grid=0)
    got, st = gpu_field(lp, sc, stats=True)
    ks = np.arange(96 * 96)
    ref, ost = orc.generate(sc, ks, stats=True)
    nd = nondegenerate(96, 96, ks)
    assert rel_l1(got[nd], ref[nd]) <= RAD_TOL
    assert abs(st[0] / ost[0] - 1) < 1e-3 and st[4] == 0  # one cell: the walk never steps


def test_grid_cuts_tentative_collisions(lp, orc):
    """On the CT-like phantom a 16^3 grid cuts the tentative collisions many
    times over; each estimator matches the oracle's of the same kind (their
    agreement in expectation is pinned on the oracle)."""
    sc = S.config(2, M=128, N=128, spp=8, grid=16)
    a, sa = gpu_field(lp, sc.with_params(grid=0), stats=True)
    b, sb = gpu_field(lp, sc, stats=True)
    print(f"tentative collisions: global {sa[0]}, grid {sb[0]} ({sa[0] / sb[0]:.1f}x); "
          f"shadow steps {sa[1]} -> {sb[1]}; cell steps {sb[4]}")
    assert sa[0] > 5 * sb[0] and sa[2] > 0
    ks = S.random_rays(128, 128, 1500, 9)
    assert rel_l1(a[ks], orc.generate(sc.with_params(grid=0), ks)) <= RAD_TOL
    assert rel_l1(b[ks], orc.generate(sc, ks)) <= RAD_TOL


def test_row_slabs_bit_identical(lp):
    sc = S.config(1, M=64, N=64, spp=4)
    vol, med, light, prm, _ = lp.device_scene(sc)
    full = lp.generate(vol, med, light, prm)
    part = torch.zeros_like(full)
    for a, b in [(0, 21), (21, 22), (22, 22), (22, 64), (64, 64)]:  # (empty ranges write nothing)
        lp.generate(vol, med, light, dataclasses.replace(prm, row_begin=a, row_end=b), out=part)
    torch.cuda.synchronize()
    assert torch.equal(full, part)
    # an empty range leaves the output as it was, with and without the kept sample radiance
    sentinel = torch.full_like(full, -7.0)
    srad = torch.full((64, 64, 4, 3), -7.0, device="cuda")
    lp.generate(vol, med, light, dataclasses.replace(prm, row_begin=30, row_end=30), out=sentinel,
                sample_radiance=srad)
    torch.cuda.synchronize()
    assert bool((sentinel == -7.0).all()) and bool((srad == -7.0).all())


def test_bricked_equals_linear(lp, orc):
    """The 8^3 brick-major layout reads exactly the same voxels."""
    v = S.phantom_volume(64, 1234, 8)
    lin = S.Volume(v.reshape(-1), S.U16, (64, 64, 64), 0, 24.0, 3024.0)
    brk = S.Volume(S.brick_layout(v, 8), S.U16, (64, 64, 64), 8, 24.0, 3024.0)
    sc = S.config(2, M=128, N=128, spp=4)
    a = gpu_field(lp, sc.replace(volume=lin))
    b = gpu_field(lp, sc.replace(volume=brk))
    assert np.array_equal(a, b)
    ks = S.random_rays(128, 128, 1500, 3)
    ref = orc.generate(sc.replace(volume=brk), ks)
    assert rel_l1(b[ks], ref) <= RAD_TOL


def test_white_furnace(lp):
    sc = S.config(1, M=64, N=64, spp=8, max_bounces=1000)
    lut = sc.medium.lut.copy()
    lut[:, :3] = 1.0
    sc = sc.replace(medium=S.Medium(lut, 40.0),
                    light=dataclasses.replace(sc.light, radiance=(0, 0, 0), env=(1.0, 1.0, 1.0)))
    got = gpu_field(lp, sc)
    ks = np.arange(64 * 64)
    assert np.all(got[nondegenerate(64, 64, ks)] == 1.0)


def test_vacuum_and_linearity(lp):
    sc = S.config(1, M=32, N=32, spp=4)
    vac = gpu_field(lp, sc.replace(medium=S.Medium(sc.medium.lut, 0.0),
                                   light=dataclasses.replace(sc.light, env=(0.25, 0.5, 1.0))))
    nd = nondegenerate(32, 32, np.arange(32 * 32))
    assert np.all(vac[nd] == np.array([0.25, 0.5, 1.0]))
    a = gpu_field(lp, sc)
    b = gpu_field(lp, sc.replace(light=dataclasses.replace(sc.light, radiance=(2.0, 2.0, 2.0))))
    assert np.array_equal(b, 2 * a)


def sf_chords(orc, M, N):
    """FP64 SF origins on S and unit directions of every ray k = i*N + j."""
    R = math.sqrt(3.0)
    o = orc.sf_points(M) * R
    d = orc.sf_points(N) * R
    i, j = np.divmod(np.arange(M * N), N)
    v = d[j] - o[i]
    n = np.linalg.norm(v, axis=1, keepdims=True)
    return o[i], v / np.where(n > 0, n, 1.0)


def chord_misses(o, d, lo, hi):
    """True where o + t d (t >= 0) misses the box [lo, hi]^3 (FP64 slabs)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t1, t2 = (lo - o) / d, (hi - o) / d
    tn = np.maximum(np.nanmax(np.minimum(t1, t2), axis=1), 0.0)
    tf = np.nanmin(np.maximum(t1, t2), axis=1)
    return ~(tn < tf)


@pytest.mark.parametrize("jitter", [1, 0])
def test_rays_missing_the_box(lp, orc, jitter):
    """Rays whose every sample misses the volume box are finished at once:
    each of them holds the FP32 sum of spp environment samples / spp, the
    value the per-sample loop adds up.  Rays near the box's silhouette take
    the per-sample path; all rays match the oracle.  (A box of half size, so
    that about half of the chords miss it.)"""
    M = N = 64
    spp = 8
    sc = S.config(1, M=M, N=N, spp=spp, jitter=jitter)
    sc = sc.replace(volume=dataclasses.replace(sc.volume, box_min=(-0.5, -0.5, -0.5), box_max=(0.5, 0.5, 0.5)),
                    light=dataclasses.replace(sc.light, env=(0.3, 0.2, 0.1)))
    got = gpu_field(lp, sc)
    o, d = sf_chords(orc, M, N)
    pad = 2.0 * math.sqrt(3.0) / math.sqrt(M) * 1.01 + 1e-4 if jitter else 1e-4
    miss = chord_misses(o, d, -0.5 - pad, 0.5 + pad)
    ks = nondegenerate(M, N, np.arange(M * N))
    miss_ks = ks[miss[ks]]
    assert 0.2 * len(ks) < len(miss_ks) < 0.9 * len(ks)
    acc = np.zeros(3, np.float32)
    for _ in range(spp):
        acc = acc + np.array([0.3, 0.2, 0.1], np.float32)
    want = (acc / np.float32(spp)).astype(np.float64)
    assert np.array_equal(got[miss_ks], np.broadcast_to(want, (len(miss_ks), 3)))
    ref = orc.generate(sc, ks)
    assert rel_l1(got[ks], ref) <= RAD_TOL


@pytest.mark.parametrize("dtype,bound", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_half_storage(lp, orc, dtype, bound):
    """FP16/BF16 storage rounds the FP32 mean once (round to nearest even)."""
    sc = S.config(1)
    f32 = gpu_field(lp, sc)
    low = gpu_field(lp, sc, dtype=dtype)
    nz = f32 > (6.2e-5 if dtype == "f16" else 1e-30)
    assert np.all(np.abs(low[nz] - f32[nz]) <= bound * np.abs(f32[nz]))
    ref_dt = torch.tensor(f32.astype(np.float32)).to(torch.float16 if dtype == "f16" else torch.bfloat16)
    assert np.array_equal(low.astype(np.float32), ref_dt.float().numpy())
    ks = nondegenerate(256, 256, S.random_rays(256, 256, 3000, 8))
    ref = orc.generate(sc, ks)
    print(f"{dtype}: rel L1 vs FP64 oracle {rel_l1(low[ks], ref):.3e} (FP32: {rel_l1(f32[ks], ref):.3e})")


def test_frozen_sampling(lp, orc):
    sc = S.config(1, M=64, N=64, spp=8)
    base = gpu_field(lp, sc)
    same = gpu_field(lp, sc, sample=S.Medium(sc.medium.lut.copy(), sc.medium.scale))
    assert np.array_equal(base, same)  # all weights are exactly 1 at theta_0
    sig = orc.majorant(sc.medium, sc.params)
    sc_fixed = sc.with_params(majorant=sig)
    pert = S.Medium(np.clip(sc.medium.lut + 0.05, 0, 1).astype(np.float32), sc.medium.scale * 1.1)
    got = gpu_field(lp, sc_fixed.replace(medium=pert), sample=sc.medium)
    ks = nondegenerate(64, 64, np.arange(64 * 64))
    ref = orc.generate(sc_fixed.replace(medium=pert), ks, sample_medium=sc.medium)
    assert rel_l1(got[ks], ref) <= RAD_TOL


# ------------------------------------------------------------------ lookup
def lookup_case(lp, orc, M, N, views, W, H, K, dtype="f32", seed=0, pix=None):
    rng = np.random.default_rng(seed)
    lf32 = rng.uniform(0.0, 1.0, (M, N, 3)).astype(np.float32)
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    lf = torch.from_numpy(lf32).to(tdt).cuda()
    sc = S.config(2, M=M, N=N, views=views, width=W, height=H)
    prm = lp.GenParams(M=M, N=N, radius=sc.params.radius)
    cams = [lp.Camera(c.eye, c.target, c.up, c.vfov) for c in sc.cams]
    img, nn = lp.lookup(lf, prm, cams, W, H, K=K, with_nn=True)
    torch.cuda.synchronize()
    g_img = img.reshape(-1, 3).cpu().numpy()
    g_nn = nn.reshape(-1, 2).cpu().numpy()
    if pix is None:
        pix = orc.all_pixels(views, W, H)
    flat = (pix[:, 0].astype(np.int64) * H + pix[:, 2]) * W + pix[:, 1]
    lf_host = lf.float().cpu().numpy()
    rgb, onn, mg = orc.lookup(lf_host, sc.params, sc.cams, W, H, K, pix)
    clear = (mg[:, 0] > 1e-4) & (mg[:, 1] > BAND) & (mg[:, 2] > 1e-3) & ((mg[:, 3] > BAND) | (K == 1))
    return g_img[flat], g_nn[flat], rgb, onn, clear, lookup_tol(M, N, lf_host)


@pytest.mark.parametrize("K", [1, 3, 5, 9])
def test_lookup_small(lp, orc, K):
    g_img, g_nn, rgb, onn, clear, tol = lookup_case(lp, orc, 256, 256, 3, 72, 40, K)
    err = np.abs(g_img[clear] - rgb[clear])
    print(f"K={K}: {(~clear).sum()} of {len(clear)} pixels inside a decision band; "
          f"max |err| {err.max():.2e} (tol {tol:.2e})")
    assert clear.mean() > 0.995
    assert np.array_equal(g_nn[clear], onn[clear])
    if K == 1:
        assert np.array_equal(g_img[clear], rgb[clear])  # nearest sampling copies the texel
    check_pixels(g_img[clear], rgb[clear], tol)
    hit = onn[:, 0] >= 0
    assert np.all(g_img[clear & ~hit] == 0.0) and np.all(g_nn[clear & ~hit] == -1)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_lookup_half_storage(lp, orc, dtype):
    g_img, g_nn, rgb, onn, clear, tol = lookup_case(lp, orc, 200, 180, 2, 48, 36, 5, dtype=dtype, seed=3)
    assert np.array_equal(g_nn[clear], onn[clear])
    check_pixels(g_img[clear], rgb[clear], tol)


@pytest.mark.parametrize("M,N", [(65535, 1024), (1024, 65535)])
@pytest.mark.parametrize("K", [1, 5])
def test_lookup_largest_point_sets(lp, orc, M, N, K):
    """The largest SF sets the lookup takes (65535 points, the top zones of
    the inverse mapping), for the origins and for the directions, with the
    other set small: 3000 sampled pixels of 2 views of 640 x 360."""
    rng = np.random.default_rng(71)
    V, W, H = 2, 640, 360
    pix = np.stack([rng.integers(0, V, 3000), rng.integers(0, W, 3000), rng.integers(0, H, 3000)], 1)
    g_img, g_nn, rgb, onn, clear, tol = lookup_case(lp, orc, M, N, V, W, H, K, seed=72, pix=pix.astype(np.int32))
    assert clear.mean() > 0.99
    assert np.array_equal(g_nn[clear], onn[clear])
    if K == 1:
        assert np.array_equal(g_img[clear], rgb[clear])
    check_pixels(g_img[clear], rgb[clear], tol)


def test_lookup_c2_full_size_sampled(lp, orc):
    """32 views of 1920 x 1080 over an N = 2048 light field (the benchmark's
    lookup), checked on 6000 sampled pixels."""
    rng = np.random.default_rng(9)
    V, W, H = 32, 1920, 1080
    pix = np.stack([rng.integers(0, V, 6000), rng.integers(0, W, 6000), rng.integers(0, H, 6000)], 1)
    g_img, g_nn, rgb, onn, clear, tol = lookup_case(lp, orc, 2048, 2048, V, W, H, 5, pix=pix.astype(np.int32))
    assert clear.mean() > 0.99
    assert np.array_equal(g_nn[clear], onn[clear])
    check_pixels(g_img[clear], rgb[clear], tol)


@pytest.mark.parametrize("M,N,K", [(96, 80, 5), (64, 64, 5), (64, 64, 1), (96, 80, 9), (64, 64, 3), (96, 80, 2)])
def test_lookup_adjoint(lp, orc, M, N, K):
    V, W, H = 2, 40, 30
    sc = S.config(1, M=M, N=N, views=V, width=W, height=H)
    prm = lp.GenParams(M=M, N=N, radius=sc.params.radius)
    cams = [lp.Camera(c.eye, c.target, c.up, c.vfov) for c in sc.cams]
    rng = np.random.default_rng(4)
    dimg = rng.standard_normal((V, H, W, 3)).astype(np.float32)
    d_lf = lp.lookup_adjoint(torch.from_numpy(dimg).cuda(), prm, cams, K)
    torch.cuda.synchronize()
    pix = orc.all_pixels(V, W, H)
    flat = (pix[:, 0].astype(np.int64) * H + pix[:, 2]) * W + pix[:, 1]
    ref = orc.lookup_adjoint(sc.params, sc.cams, W, H, K, pix, dimg.reshape(-1, 3)[flat].astype(np.float64))
    got = d_lf.reshape(-1).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)


def tile_rays_disc(cam, W, H, R):
    """disc / R^2 of the sphere test for the centre pixel of every 8x8 tile
    (the lookup's pinhole camera, FP64): [H // 8, W // 8]."""
    eye, tgt, up = (np.asarray(x, np.float64) for x in (cam.eye, cam.target, cam.up))
    f = (tgt - eye) / np.linalg.norm(tgt - eye)
    rt = np.cross(f, up)
    rt /= np.linalg.norm(rt)
    u = np.cross(rt, f)
    th = math.tan(0.5 * cam.vfov)
    ty, tx = np.meshgrid(np.arange(H // 8), np.arange(W // 8), indexing="ij")
    ndx = (2.0 * (tx * 8 + 4.0) / W - 1.0) * th * W / H
    ndy = (1.0 - 2.0 * (ty * 8 + 4.0) / H) * th
    d = f + rt * ndx[..., None] + u * ndy[..., None]
    d /= np.linalg.norm(d, axis=-1)[..., None]
    b = d @ eye
    return (b * b - (eye @ eye - R * R)) / (R * R)


def full_resolution_adjoint(lp, orc, c, M, W, H, K, n_inf=0):
    """d_lf from the GPU and the oracle for one view of workload c at full
    resolution: the adjoint image is nonzero on the decided pixels of 240
    random 8x8 tiles and of up to 60 tiles next to the silhouette; n_inf of
    those pixels carry +inf in channel 0."""
    sc = S.config(c, M=M, N=M, views=1, width=W, height=H)
    R = sc.params.radius
    prm = lp.GenParams(M=M, N=M, radius=R)
    cams = [lp.Camera(x.eye, x.target, x.up, x.vfov) for x in sc.cams]
    rng = np.random.default_rng(11)
    mask = np.zeros((H, W), bool)
    for tx, ty in zip(rng.integers(0, W // 8, 240), rng.integers(0, H // 8, 240)):
        mask[8 * ty:8 * ty + 8, 8 * tx:8 * tx + 8] = True
    disc = tile_rays_disc(sc.cams[0], W, H, R)
    edge = np.argwhere((disc > 0.0) & (disc < 0.02))
    for ty, tx in edge[rng.permutation(len(edge))[:60]]:
        mask[8 * ty:8 * ty + 8, 8 * tx:8 * tx + 8] = True
    pix = orc.all_pixels(1, W, H)
    sel = pix[mask.reshape(-1)[pix[:, 2].astype(np.int64) * W + pix[:, 1]]]
    # pixels inside an FP32 decision band of the neighbour search (either
    # neighbour set may differ from FP64) keep a zero adjoint
    _, onn, mg = orc.lookup(np.zeros((M, M, 3), np.float32), sc.params, sc.cams, W, H, K, sel)
    clear = (mg[:, 0] > 1e-4) & (mg[:, 1] > BAND) & (mg[:, 2] > 1e-3) & ((mg[:, 3] > BAND) | (K == 1))
    assert clear.mean() > 0.97
    keep, knn = sel[clear], onn[clear]
    vals = rng.standard_normal((len(keep), 3)).astype(np.float32)
    if n_inf:
        hits = np.nonzero(knn[:, 0] >= 0)[0]
        vals[rng.choice(hits, n_inf, replace=False), 0] = np.inf
    dimg = np.zeros((1, H, W, 3), np.float32)
    dimg[0, keep[:, 2], keep[:, 1]] = vals
    d_lf = lp.lookup_adjoint(torch.from_numpy(dimg).cuda(), prm, cams, K)
    torch.cuda.synchronize()
    ref = orc.lookup_adjoint(sc.params, sc.cams, W, H, K, keep, vals.astype(np.float64))
    got = d_lf.reshape(-1).cpu().numpy().astype(np.float64)
    return got, ref


@pytest.mark.parametrize("c,M,W,H,K", [(5, 1024, 512, 512, 5), (2, 2048, 1920, 1080, 5),
                                       (2, 2048, 1920, 1080, 1), (2, 2048, 1920, 1080, 9),
                                       (5, 1024, 512, 512, 3)])
def test_lookup_adjoint_full_resolution(lp, orc, c, M, W, H, K):
    """At the workloads' view sizes the 64 pixels of a wave share a handful of
    neighbours, and the scatter runs as a dense contraction per wave (MFMA)
    over the wave's distinct origin and direction texels; waves with more
    distinct texels (K = 9 always) take the per-pair path.  Silhouette
    tiles are where front and back hits meet the same SF point and
    degenerate pairs occur; the oracle transposes the selected pixels only
    (the other pixels still enter the waves' neighbour dictionaries)."""
    got, ref = full_resolution_adjoint(lp, orc, c, M, W, H, K)
    assert np.count_nonzero(ref) > 1000
    # the lookup's bar: FP32 view rays move each tent weight by ~1e-6 / r
    r = math.sqrt(4 * math.pi / M)
    assert np.linalg.norm(got - ref) <= LOOKUP_C / r * np.linalg.norm(ref)
    # texels no selected pixel reaches stay exactly zero
    assert np.all(got[ref == 0.0] == 0.0)


def test_lookup_adjoint_infinite_values(lp, orc):
    """A wave holding a non-finite adjoint value takes the per-pair path: the
    infinities reach exactly the texels their pixels weight, as in the
    oracle, and no NaN appears (in the dense contraction a zero weight times
    an infinite value would spread NaN over the wave's other texels)."""
    M = 1024
    got, ref = full_resolution_adjoint(lp, orc, 5, M, 512, 512, 5, n_inf=6)
    inf = np.isinf(ref)
    assert 6 <= inf.sum() and not np.isnan(ref).any()
    assert np.array_equal(np.isinf(got), inf) and not np.isnan(got).any()
    fin = ~inf
    r = math.sqrt(4 * math.pi / M)
    assert np.linalg.norm(got[fin] - ref[fin]) <= LOOKUP_C / r * np.linalg.norm(ref[fin])


# ------------------------------------------------- upper-hemisphere origins
def test_generate_stored_rows(lp, orc):
    """origin_rows = M/2 writes the first half of the full field, bit for bit,
    as a [M/2][N][3] array; row slabs inside it split the same work."""
    sc = S.config(1, M=96, N=80, spp=4)
    full = gpu_field(lp, sc).reshape(96, 80, 3)
    half_sc = sc.with_params(origin_rows=48)
    vol, med, light, prm, _ = lp.device_scene(half_sc)
    assert prm.rows == 48
    lf = lp.generate(vol, med, light, prm)
    assert tuple(lf.shape) == (48, 80, 3)
    torch.cuda.synchronize()
    assert np.array_equal(lf.cpu().numpy().astype(np.float64), full[:48])
    slab = torch.full_like(lf, -1.0)
    for r0, r1 in ((0, 17), (17, 48)):
        lp.generate(vol, med, light, dataclasses.replace(prm, row_begin=r0, row_end=r1), out=slab)
    assert torch.equal(slab, lf)
    ks = np.arange(48 * 80)
    ref = orc.generate(half_sc, ks)
    assert rel_l1(lf.reshape(-1, 3).double().cpu().numpy(), ref) <= RAD_TOL
    with pytest.raises(lp.LumiPathError):
        lp.generate(vol, med, light, dataclasses.replace(prm, row_end=49), out=lf)


def stored_rows_case(lp, orc, M, N, rows, K, dtype="f32", seed=5):
    R = math.sqrt(3.0)
    rng = np.random.default_rng(seed)
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
    lf = torch.from_numpy(rng.uniform(0.0, 1.0, (rows, N, 3)).astype(np.float32)).to(tdt).cuda()
    cams = S.seam_cameras(R)
    W, H = 64, 48
    prm = lp.GenParams(M=M, N=N, radius=R, origin_rows=rows)
    img, nn = lp.lookup(lf, prm, [lp.Camera(c.eye, c.target, c.up, c.vfov) for c in cams], W, H, K=K,
                        with_nn=True)
    torch.cuda.synchronize()
    pix = orc.all_pixels(len(cams), W, H)
    flat = (pix[:, 0].astype(np.int64) * H + pix[:, 2]) * W + pix[:, 1]
    lf_host = lf.float().cpu().numpy()
    rgb, onn, mg = orc.lookup(lf_host, S.Params(M=M, N=N, radius=R, origin_rows=rows), cams, W, H, K, pix)
    clear = (mg[:, 0] > 1e-4) & (mg[:, 1] > BAND) & (mg[:, 2] > 1e-3) & ((mg[:, 3] > BAND) | (K == 1))
    return (img.reshape(-1, 3).cpu().numpy()[flat], nn.reshape(-1, 2).cpu().numpy()[flat], rgb, onn, clear,
            lookup_tol(M, N, lf_host), cams, W, H)


@pytest.mark.parametrize("M,N,K", [(300, 256, 1), (300, 256, 5), (256, 256, 5), (300, 256, 9)])
def test_lookup_stored_rows(lp, orc, M, N, K):
    rows = M // 2
    g_img, g_nn, rgb, onn, clear, tol, _, _, _ = stored_rows_case(lp, orc, M, N, rows, K)
    assert clear.mean() > 0.99
    assert np.array_equal(g_nn[clear], onn[clear])
    uncovered = clear & (onn[:, 0] >= 0) & np.all(rgb == 0.0, 1)
    assert uncovered.sum() > 100        # the views see origins that are not stored
    assert np.all(g_img[uncovered] == 0.0)
    if K == 1:
        assert np.array_equal(g_img[clear], rgb[clear])
    check_pixels(g_img[clear], rgb[clear], tol)


@pytest.mark.parametrize("K", [1, 5])
def test_lookup_adjoint_stored_rows(lp, orc, K):
    M, N, rows = 96, 80, 48
    R = math.sqrt(3.0)
    cams = S.seam_cameras(R)
    V, W, H = len(cams), 40, 30
    prm = lp.GenParams(M=M, N=N, radius=R, origin_rows=rows)
    rng = np.random.default_rng(6)
    dimg = rng.standard_normal((V, H, W, 3)).astype(np.float32)
    d_lf = lp.lookup_adjoint(torch.from_numpy(dimg).cuda(), prm,
                             [lp.Camera(c.eye, c.target, c.up, c.vfov) for c in cams], K)
    torch.cuda.synchronize()
    assert tuple(d_lf.shape) == (rows, N, 3)
    pix = orc.all_pixels(V, W, H)
    flat = (pix[:, 0].astype(np.int64) * H + pix[:, 2]) * W + pix[:, 1]
    ref = orc.lookup_adjoint(S.Params(M=M, N=N, radius=R, origin_rows=rows), cams, W, H, K, pix,
                             dimg.reshape(-1, 3)[flat].astype(np.float64))
    got = d_lf.reshape(-1).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)


@pytest.mark.parametrize("K,dtype,rows,N", [(5, "f32", 0, 256), (1, "f32", 0, 256), (5, "f16", 0, 256),
                                            (9, "bf16", 0, 256), (5, "f32", 128, 256), (1, "f32", 128, 256),
                                            (3, "f32", 0, 256), (5, "f32", 0, 192), (5, "bf16", 128, 320)])
def test_lookup_l2_fused(lp, K, dtype, rows, N):
    """lf_lookup_l2 writes the forward views bit for bit and adds the
    transpose of (views - target) to d_lf, as lookup, subtraction and
    lookup_adjoint do separately (to float-atomic rounding); also with only
    the upper-hemisphere origin rows stored, with fewer neighbours than the
    kernel's five slots, and with two different point sets (no degenerate
    pairs: every wave blends separably)."""
    M = 256
    V, W, H = 3, 96, 64
    sc = S.config(1, M=M, N=N, views=V, width=W, height=H, origin_rows=rows)
    if rows:
        sc = sc.replace(cams=S.seam_cameras(math.sqrt(3.0))[:V])
    vol, med, light, prm, cams = lp.device_scene(sc)
    lf = lp.generate(vol, med, light, prm, dtype=dtype)
    torch.manual_seed(0)
    target = torch.rand((V, H, W, 3), device="cuda")
    img_ref = lp.lookup(lf, prm, cams, W, H, K)
    d_ref = lp.lookup_adjoint(img_ref - target, prm, cams, K)
    img, d_lf = lp.lookup_l2(lf, prm, cams, target, K)
    torch.cuda.synchronize()
    assert torch.equal(img, img_ref)
    a, b = d_lf.double(), d_ref.double()
    assert float((a - b).norm()) <= 1e-5 * float(b.norm())


# ------------------------------------------------------------------ adjoint
def grad_scene():
    sc = S.config(1, M=48, N=48, spp=6, max_bounces=3, g=0.3)
    lut = (0.05 + 0.9 * sc.medium.lut).astype(np.float32)
    lut[0, 3] = 0.0
    return sc.replace(medium=S.Medium(lut, 25.0), light=dataclasses.replace(sc.light, env=(0.3, 0.2, 0.1)))


def test_backward_matches_oracle_gradient(lp, orc):
    sc = grad_scene()
    M = N = 48
    rng = np.random.default_rng(12)
    ks = nondegenerate(M, N, S.random_rays(M, N, 600, 7))
    adj = rng.standard_normal((len(ks), 3))
    d_lf = np.zeros((M * N, 3), np.float32)
    d_lf[ks] = adj
    vol, med, light, prm, _ = lp.device_scene(sc)
    d_lut, d_scale = lp.generate_backward(vol, med, light, prm, torch.from_numpy(d_lf).cuda())
    torch.cuda.synchronize()
    g_lut = d_lut.cpu().numpy().astype(np.float64)
    o_lut, o_scale = orc.gradient(sc, ks, d_lf[ks].astype(np.float64))
    err = np.linalg.norm(g_lut - o_lut) / np.linalg.norm(o_lut)
    print(f"adjoint vs oracle gradient: {err:.2e}, dscale {float(d_scale[0]):.6g} vs {o_scale:.6g}")
    assert err <= 1e-3
    assert abs(float(d_scale[0]) - o_scale) <= 1e-3 * abs(o_scale)


def test_backward_from_stored_sample_radiance(lp, orc):
    """generate() keeps each sample's radiance (their in-order FP32 mean is
    the field); generate_backward() given that buffer skips its first pass
    and returns the same gradient."""
    sc = grad_scene()
    M = N = 48
    spp = sc.params.spp
    vol, med, light, prm, _ = lp.device_scene(sc)
    srad = torch.full((M, N, spp, 3), float("nan"), dtype=torch.float32, device="cuda")
    lf = lp.generate(vol, med, light, prm, sample_radiance=srad)
    torch.cuda.synchronize()
    field = lf.reshape(-1, 3).cpu().numpy()
    sr = srad.reshape(M * N, spp, 3).cpu().numpy()
    written = ~np.isnan(sr[:, 0, 0])
    assert written.sum() > 0.5 * M * N
    acc = np.zeros((M * N, 3), np.float32)
    for s_ in range(spp):
        acc = acc + sr[:, s_]
    assert np.array_equal((acc / np.float32(spp))[written], field[written])
    rng = np.random.default_rng(15)
    adj = rng.standard_normal((M * N, 3)).astype(np.float32)
    adj[np.arange(M) * (N + 1)] = 0.0
    d = torch.from_numpy(adj).cuda()
    a_lut, a_s = lp.generate_backward(vol, med, light, prm, d)
    b_lut, b_s = lp.generate_backward(vol, med, light, prm, d, sample_radiance=srad)
    torch.cuda.synchronize()
    a = np.concatenate([a_lut.cpu().numpy().reshape(-1), a_s.cpu().numpy()]).astype(np.float64)
    b = np.concatenate([b_lut.cpu().numpy().reshape(-1), b_s.cpu().numpy()]).astype(np.float64)
    assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(a)


@pytest.mark.parametrize("spp,ranges", [(8, 1), (16, 2), (32, 4)])
def test_mean_over_sample_ranges(lp, spp, ranges):
    """The texel is the FP32 sum of each range of spp / R consecutive
    samples in order, then of the R range sums in order, divided by spp
    (R = 4 from 32 samples, 2 from 16); the kept per-sample radiance shows
    each sample's value."""
    M = N = 64
    sc = S.config(1, M=M, N=N, spp=spp)
    vol, med, light, prm, _ = lp.device_scene(sc)
    srad = torch.full((M, N, spp, 3), float("nan"), dtype=torch.float32, device="cuda")
    lf = lp.generate(vol, med, light, prm, sample_radiance=srad)
    torch.cuda.synchronize()
    field = lf.reshape(-1, 3).cpu().numpy()
    sr = srad.reshape(M * N, spp, 3).cpu().numpy()
    whole = ~np.isnan(sr).any(axis=(1, 2))
    assert whole.sum() > 0.3 * M * N
    n = spp // ranges
    total = np.zeros((M * N, 3), np.float32)
    for r_ in range(ranges):
        part = np.zeros((M * N, 3), np.float32)
        for s_ in range(r_ * n, (r_ + 1) * n):
            part = part + sr[:, s_]
        total = part if r_ == 0 else total + part
    assert np.array_equal((total / np.float32(spp))[whole], field[whole])
    # the same field without keeping the samples, and split by rows
    assert np.array_equal(lp.generate(vol, med, light, prm).reshape(-1, 3).cpu().numpy(), field)
    half = dataclasses.replace(prm, row_begin=M // 2, row_end=M)
    out = torch.zeros_like(lf)
    lp.generate(vol, med, light, half, out=out)
    assert np.array_equal(out.reshape(-1, 3).cpu().numpy()[M // 2 * N:], field[M // 2 * N:])


def test_backward_matches_finite_differences(lp, orc):
    """Central differences (h = 1e-3) of the GPU forward in frozen sampling."""
    sc = grad_scene()
    M = N = 48
    sig = orc.majorant(sc.medium, sc.params)
    sc = sc.with_params(majorant=sig)
    rng = np.random.default_rng(13)
    adj = rng.standard_normal((M * N, 3))
    adj[np.arange(M) * (N + 1)] = 0.0
    vol, med, light, prm, _ = lp.device_scene(sc)
    d_lut, d_scale = lp.generate_backward(vol, med, light, prm, torch.from_numpy(adj.astype(np.float32)).cuda())
    g = np.concatenate([d_lut.cpu().numpy().reshape(-1), d_scale.cpu().numpy()]).astype(np.float64)
    theta0 = sc.medium
    smp = lp.Medium(torch.from_numpy(theta0.lut).cuda(), theta0.scale)

    def loss(lut, scale):
        m = lp.Medium(torch.from_numpy(lut).cuda(), scale)
        L = lp.generate(vol, m, light, prm, sample=smp).double().cpu().numpy().reshape(-1, 3)
        return float((L * adj).sum())

    h = 1e-3
    fd = np.zeros_like(g)
    touched = np.argwhere(np.abs(g[:-1].reshape(-1, 4)) > 1e-4 * np.abs(g).max())
    for e, c in touched:
        lp_, lm = theta0.lut.copy(), theta0.lut.copy()
        lp_[e, c] += h
        lm[e, c] -= h
        fd[4 * e + c] = (loss(lp_, theta0.scale) - loss(lm, theta0.scale)) / (float(lp_[e, c]) - float(lm[e, c]))
    fd[-1] = (loss(theta0.lut, theta0.scale + h) - loss(theta0.lut, theta0.scale - h)) / (2 * h)
    mask = np.zeros_like(g, bool)
    mask[[4 * e + c for e, c in touched]] = True
    mask[-1] = True
    err = np.linalg.norm(fd[mask] - g[mask]) / np.linalg.norm(g[mask])
    print(f"adjoint vs central differences on {mask.sum()} coordinates: {err:.2e}")
    assert err <= 1e-2


def test_backward_with_grid_matches_finite_differences(lp, orc):
    """As above with the majorant grid, built from the reference medium in
    both the frozen-sampling forward and the adjoint."""
    sc = grad_scene()
    assert sc.params.grid > 0 and sc.params.majorant == 0.0
    M = N = 48
    rng = np.random.default_rng(14)
    adj = rng.standard_normal((M * N, 3))
    adj[np.arange(M) * (N + 1)] = 0.0
    vol, med, light, prm, _ = lp.device_scene(sc)
    d_lut, d_scale = lp.generate_backward(vol, med, light, prm, torch.from_numpy(adj.astype(np.float32)).cuda())
    g = np.concatenate([d_lut.cpu().numpy().reshape(-1), d_scale.cpu().numpy()]).astype(np.float64)
    theta0 = sc.medium
    smp = lp.Medium(torch.from_numpy(theta0.lut).cuda(), theta0.scale)

    def loss(lut, scale):
        m = lp.Medium(torch.from_numpy(lut).cuda(), scale)
        L = lp.generate(vol, m, light, prm, sample=smp).double().cpu().numpy().reshape(-1, 3)
        return float((L * adj).sum())

    h = 1e-3
    fd = np.zeros_like(g)
    touched = np.argwhere(np.abs(g[:-1].reshape(-1, 4)) > 1e-4 * np.abs(g).max())
    for e, c in touched:
        lp_, lm = theta0.lut.copy(), theta0.lut.copy()
        lp_[e, c] += h
        lm[e, c] -= h
        fd[4 * e + c] = (loss(lp_, theta0.scale) - loss(lm, theta0.scale)) / (float(lp_[e, c]) - float(lm[e, c]))
    fd[-1] = (loss(theta0.lut, theta0.scale + h) - loss(theta0.lut, theta0.scale - h)) / (2 * h)
    mask = np.zeros_like(g, bool)
    mask[[4 * e + c for e, c in touched]] = True
    mask[-1] = True
    err = np.linalg.norm(fd[mask] - g[mask]) / np.linalg.norm(g[mask])
    print(f"grid adjoint vs central differences on {mask.sum()} coordinates: {err:.2e}")
    assert err <= 1e-2


@pytest.mark.parametrize("keep_samples", [False, True])
def test_autograd_pipeline(lp, orc, keep_samples):
    """Differentiation workload, reduced: LightFieldFn -> LookupFn -> L2 loss;
    the LUT gradient equals the oracle's chain (lookup transpose, then the
    path-replay gradient) on the same views, with the adjoint tracing each
    sample twice or reading the radiance the forward kept."""
    M = N = 64
    V, W, H, K = 3, 48, 40, 5
    sc = S.config(5, M=M, N=N, spp=8, views=V, width=W, height=H)
    vol, med, light, prm, cams = lp.device_scene(sc)
    tgt = S.target_medium(sc)
    # targets and their oracle counterparts from the oracle's own forward
    ks = np.arange(M * N)
    lf_t = orc.generate(sc.replace(medium=tgt), ks).astype(np.float32)
    pix = orc.all_pixels(V, W, H)
    flat = (pix[:, 0].astype(np.int64) * H + pix[:, 2]) * W + pix[:, 1]
    t_rgb, _, _ = orc.lookup(lf_t, sc.params, sc.cams, W, H, K, pix)
    target = np.zeros((V * H * W, 3), np.float32)
    target[flat] = t_rgb
    lut = med.lut.clone().requires_grad_(True)
    scale = torch.tensor(float(med.scale), requires_grad=True)
    lf = lp.LightFieldFn.apply(lut, scale, vol, light, prm, keep_samples)
    img = lp.LookupFn.apply(lf, prm, cams, W, H, K)
    loss = ((img - torch.from_numpy(target.reshape(V, H, W, 3)).cuda()) ** 2).sum()
    loss.backward()
    g_lut = lut.grad.cpu().numpy().astype(np.float64)
    # oracle chain
    lf_o = orc.generate(sc, ks)
    o_rgb, _, _ = orc.lookup(lf_o.astype(np.float32), sc.params, sc.cams, W, H, K, pix)
    dimg = 2 * (o_rgb - target[flat])
    d_lf = orc.lookup_adjoint(sc.params, sc.cams, W, H, K, pix, dimg).reshape(-1, 3)
    rows = np.nonzero(np.abs(d_lf).sum(1))[0]
    o_lut, o_scale = orc.gradient(sc, rows, d_lf[rows])
    err = np.linalg.norm(g_lut - o_lut) / np.linalg.norm(o_lut)
    print(f"pipeline gradient vs oracle chain: {err:.2e}; dscale {float(scale.grad):.5g} vs {o_scale:.5g}")
    assert err <= 1e-2
    assert abs(float(scale.grad) - o_scale) <= 1e-2 * abs(o_scale)
