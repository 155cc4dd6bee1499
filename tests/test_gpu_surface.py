"""GPU isosurface variant (lf_generate / lf_render_views with surface = 1)
against the oracle: first crossing by half-voxel march and bisection,
Lambertian next-event estimation and cosine-weighted bounces."""
import dataclasses
import math

import numpy as np
import pytest
import torch

import lfsynth as S

pytestmark = pytest.mark.gpu

ISO = 1024.0 - 500.0   # the CT phantom's body outline (air -1000 HU, body -100..300 HU)


@pytest.fixture(scope="module")
def lp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1903_03837_amd as lp
    lp.library()
    return lp


def rel_l1(got, ref):
    return float(np.abs(got - ref).sum() / np.abs(ref).sum())


def surface_scene(M=48, spp=8, **over):
    sc = S.config(2, vol_n=64, M=M, N=M, spp=spp, max_bounces=4, **over)
    lut = sc.medium.lut.copy()
    lut[:, :3] = np.clip(lut[:, :3], 0.2, 0.9)
    return dataclasses.replace(sc, medium=S.Medium(lut, sc.medium.scale),
                               light=dataclasses.replace(sc.light, env=(0.05, 0.05, 0.08))).with_params(
        surface=1, iso=ISO)


@pytest.mark.parametrize("G", [0, 5])
def test_surface_generate_matches_oracle(lp, orc, G):
    sc = surface_scene(grid=G)
    vol, med, light, prm, _ = lp.device_scene(sc)
    st = torch.zeros(5, dtype=torch.int64, device="cuda")
    lf = lp.generate(vol, med, light, prm, stats=st)
    torch.cuda.synchronize()
    got = lf.reshape(-1, 3).double().cpu().numpy()
    ks = np.arange(48 * 48)
    nd = ks[(ks // 48) != (ks % 48)]
    ref, ost = orc.generate(sc, nd, stats=True)
    err = rel_l1(got[nd], ref)
    s = st.cpu().numpy()
    print(f"surface G={G}: rel L1 {err:.2e}; vertices GPU {s[2]} oracle {int(ost[2])}")
    assert err <= 1e-3
    assert s[3] == ost[3] and abs(s[2] / ost[2] - 1) < 2e-3
    assert np.all(got[ks[(ks // 48) == (ks % 48)]] == 0.0)


def test_surface_views_match_oracle(lp, orc):
    sc = surface_scene(views=2, width=40, height=30, spp=8)
    vol, med, light, prm, cams = lp.device_scene(sc)
    img = lp.render_views(vol, med, light, prm, cams, 40, 30)
    torch.cuda.synchronize()
    pix = orc.all_pixels(2, 40, 30)
    ref = orc.render(sc, sc.cams, 40, 30, pix)
    got = img.cpu().numpy()[pix[:, 0], pix[:, 2], pix[:, 1]].astype(np.float64)
    err = rel_l1(got, ref)
    print(f"surface views rel L1 {err:.2e}")
    assert err <= 1e-3


def test_surface_white_furnace(lp):
    sc = surface_scene(spp=4)
    lut = sc.medium.lut.copy()
    lut[:, :3] = 1.0
    sc = dataclasses.replace(sc, medium=S.Medium(lut, 1.0),
                             light=dataclasses.replace(sc.light, radiance=(0, 0, 0), env=(1.0, 1.0, 1.0)))
    sc = sc.with_params(max_bounces=500)
    vol, med, light, prm, _ = lp.device_scene(sc)
    lf = lp.generate(vol, med, light, prm).reshape(-1, 3).cpu().numpy()
    ks = np.arange(48 * 48)
    assert np.all(lf[ks[(ks // 48) != (ks % 48)]] == 1.0)


def test_surface_unsupported_modes(lp):
    sc = surface_scene(spp=2)
    vol, med, light, prm, _ = lp.device_scene(sc)
    with pytest.raises(lp.LumiPathError):
        lp.generate_backward(vol, med, light, prm, torch.zeros((48, 48, 3), device="cuda"))
    with pytest.raises(lp.LumiPathError):
        lp.generate(vol, med, light, prm, sample=lp.Medium(med.lut.clone(), med.scale * 1.1))
