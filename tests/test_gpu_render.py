"""GPU ground-truth views (lf_render_views), mean SSIM (lf_ssim) and
CW-SSIM (lf_cw_ssim) against the oracle, and the evaluation they serve: light-field views against
path-traced references (the paper's Sec. 3 comparison, on synthetic
volumes)."""
import dataclasses
import math

import numpy as np
import pytest
import torch

import lfsynth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1903_03837_amd as lp
    lp.library()
    return lp


def rel_l1(got, ref):
    return float(np.abs(got - ref).sum() / np.abs(ref).sum())


def gpu_render(lp, sc, cams, W, H):
    vol, med, light, prm, _ = lp.device_scene(sc)
    img = lp.render_views(vol, med, light, prm, [lp.Camera(c.eye, c.target, c.up, c.vfov) for c in cams], W, H)
    torch.cuda.synchronize()
    return img.cpu().numpy()


@pytest.mark.parametrize("c,G", [(2, 5), (1, 0), (5, 8)])
def test_render_matches_oracle(lp, orc, c, G):
    """Every pixel of 3 views (ragged 8 x 8 tiles), same random streams."""
    sc = S.config(c, vol_n=64 if c == 2 else None, spp=16, views=3, width=45, height=30, grid=G)
    W, H = sc.width, sc.height
    got = gpu_render(lp, sc, sc.cams, W, H)
    pix = orc.all_pixels(3, W, H)
    ref = orc.render(sc, sc.cams, W, H, pix)
    g = got[pix[:, 0], pix[:, 2], pix[:, 1]].astype(np.float64)
    err = rel_l1(g, ref)
    print(f"c{c} G={G}: render rel L1 vs oracle {err:.2e}")
    assert err <= 1e-3
    assert np.all(np.isfinite(got))


def test_render_vacuum_is_environment(lp):
    sc = S.config(1, spp=4, views=2, width=20, height=17)
    sc = sc.replace(medium=S.Medium(sc.medium.lut, 0.0), light=dataclasses.replace(sc.light, env=(0.25, 0.5, 1.0)))
    got = gpu_render(lp, sc, sc.cams, 20, 17)
    assert np.all(got == np.array([0.25, 0.5, 1.0], np.float32))


def test_render_rejects_bad_views(lp):
    sc = S.config(1, spp=4, views=1, width=8, height=8)
    vol, med, light, prm, cams = lp.device_scene(sc)
    with pytest.raises(lp.LumiPathError):
        lp.render_views(vol, med, light, prm, [lp.Camera((3, 0, 0), (0, 0, 0), (1, 0, 0), 0.5)], 8, 8)


@pytest.mark.parametrize("shape", [(2, 37, 53), (1, 11, 11), (3, 64, 48)])
def test_ssim_matches_oracle(lp, orc, shape):
    n, H, W = shape
    rng = np.random.default_rng(H)
    a = rng.uniform(0, 1, (n, H, W, 3)).astype(np.float32)
    b = np.clip(0.8 * a + rng.normal(0, 0.15, a.shape) + 0.05, 0, 1).astype(np.float32)
    got = lp.ssim(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()).cpu().numpy()
    ref = orc.ssim(a, b)
    print(f"ssim {shape}: gpu {got} oracle {ref}")
    assert np.abs(got - ref).max() <= 2e-5
    same = lp.ssim(torch.from_numpy(a).cuda(), torch.from_numpy(a).cuda()).cpu().numpy()
    assert np.abs(same - 1.0).max() <= 1e-5


@pytest.mark.parametrize("shape", [(2, 37, 53), (1, 7, 7), (1, 64, 48), (1, 270, 480)])
def test_cw_ssim_matches_oracle(lp, shape):
    """lf_cw_ssim against the FP64 oracle (numpy FFT) on noisy copies.  Bar
    1e-6 absolute: the FP32 direct DFT of n <= 480 points rounds each
    coefficient at ~1e-6 relative, and the index is a ratio of window sums
    of such coefficients, whose errors largely cancel (measured 4e-9 to
    2e-8)."""
    from oracle import cwssim as cw
    n, H, W = shape
    rng = np.random.default_rng(H + W)
    a = rng.uniform(0, 1, (n, H, W, 3)).astype(np.float32)
    b = np.clip(0.8 * a + rng.normal(0, 0.15, a.shape) + 0.05, 0, 1).astype(np.float32)
    got = lp.cw_ssim(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()).cpu().numpy()
    ref = cw.cw_ssim(a, b)
    print(f"cw-ssim {shape}: gpu {got} oracle {ref} max |diff| {np.abs(got - ref).max():.2e}")
    assert np.abs(got - ref).max() <= 1e-6


def test_cw_ssim_closed_forms(lp):
    """On the GPU: a pair with itself gives 1; b = 2 a gives 2 * 2 / (1 + 4)
    with K = 0; a constant offset is filtered out (to FP32 rounding of the
    DC term)."""
    rng = np.random.default_rng(5)
    a = torch.from_numpy(rng.uniform(0, 1, (2, 40, 56, 3)).astype(np.float32)).cuda()
    one = lp.cw_ssim(a, a).cpu().numpy()
    scaled = lp.cw_ssim(a, 2.0 * a, data_range=0.0).cpu().numpy()
    shifted = lp.cw_ssim(a, a + 0.37).cpu().numpy()
    print(f"cw-ssim identity {one}, scaled {scaled}, offset {shifted}")
    assert np.abs(one - 1.0).max() <= 1e-6
    assert np.abs(scaled - 0.8).max() <= 1e-5
    assert np.abs(shifted - 1.0).max() <= 1e-4


def test_cw_ssim_rejects(lp):
    a = torch.zeros((1, 6, 9, 3), device="cuda")
    with pytest.raises(lp.LumiPathError):
        lp.cw_ssim(a, a)


def test_lightfield_views_converge_to_ground_truth(lp, orc):
    """Views synthesised from light fields of increasing resolution approach
    the path-traced views of the same cameras (SSIM up, error down); the
    GPU SSIM of each pair equals the oracle's SSIM of the same images."""
    from oracle import cwssim as cw
    V, W, H = 4, 96, 64
    sc = S.config(2, vol_n=128, views=V, width=W, height=H, spp=32)
    vol, med, light, prm, cams = lp.device_scene(sc)
    gt = lp.render_views(vol, med, light, dataclasses.replace(prm, spp=512), cams, W, H)
    scores, errs, cws = [], [], []
    for n in (128, 512, 2048):
        p = dataclasses.replace(prm, M=n, N=n)
        lf = lp.generate(vol, med, light, p)
        img = lp.lookup(lf, p, cams, W, H, K=5)
        ss = lp.ssim(img, gt, data_range=float(gt.max()))
        torch.cuda.synchronize()
        ref = orc.ssim(img.cpu().numpy(), gt.cpu().numpy(), float(gt.max()))
        assert np.abs(ss.cpu().numpy() - ref).max() <= 2e-5
        scores.append(float(ss.mean()))
        errs.append(float((img - gt).abs().mean() / gt.abs().mean()))
        c = lp.cw_ssim(img, gt, data_range=float(gt.max())).cpu().numpy()
        assert np.abs(c - cw.cw_ssim(img.cpu().numpy(), gt.cpu().numpy(), float(gt.max()))).max() <= 1e-4
        cws.append(float(c.mean()))
    print(f"light-field views vs ground truth: N = 128, 512, 2048 -> SSIM {scores}, CW-SSIM {cws}, "
          f"rel error {errs}")
    assert scores[0] < scores[1] < scores[2] and errs[0] > errs[1] > errs[2]
    assert cws[0] < cws[1] < cws[2]
    assert scores[2] > 0.5
