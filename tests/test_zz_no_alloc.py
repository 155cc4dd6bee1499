"""lf_lookup_static (the lookup entry point that allocates nothing and keeps
its point tables in the library's fixed device scratch) against lf_lookup,
through the C ABI, on two calls in a row, the second with smaller point sets
and views.  Forward views and nearest indices are bit-identical (the same
kernels on the same tables); the adjoint agrees to float-atomic rounding.
Inputs are seeded random light fields and adjoint images."""
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


CASES = [  # (M, N, views, W, H, K, stored origin rows): the second is smaller
    (2048, 1536, 3, 256, 192, 5, 0),
    (300, 256, 2, 96, 64, 5, 150),
]


def run_case(lp, M, N, V, W, H, K, rows, seed):
    rng = np.random.default_rng(seed)
    R = float(np.sqrt(3.0))
    sc = S.config(2, M=M, N=N, views=V, width=W, height=H)
    prm = lp.GenParams(M=M, N=N, radius=R, origin_rows=rows)
    cams = [lp.Camera(c.eye, c.target, c.up, c.vfov) for c in sc.cams]
    lf = torch.from_numpy(rng.uniform(0.0, 1.0, (prm.rows, N, 3)).astype(np.float32)).cuda()
    dimg = torch.from_numpy(rng.standard_normal((V, H, W, 3)).astype(np.float32)).cuda()
    # every output buffer exists before the call: the entry point allocates nothing
    img = torch.full((V, H, W, 3), float("nan"), device="cuda")
    nn = torch.full((V, H, W, 2), -7, dtype=torch.int32, device="cuda")
    d_lf = torch.zeros((prm.rows, N, 3), device="cuda")
    torch.cuda.synchronize()
    lp.lookup_static(lf, prm, cams, W, H, K, 0, img, nn=nn)
    lp.lookup_static(None, prm, cams, W, H, K, 1, dimg, d_lf=d_lf)
    ref_img, ref_nn = lp.lookup(lf, prm, cams, W, H, K, with_nn=True)
    ref_d = lp.lookup_adjoint(dimg, prm, cams, K)
    torch.cuda.synchronize()
    assert torch.equal(img, ref_img)
    assert torch.equal(nn, ref_nn)
    a, b = d_lf.double(), ref_d.double()
    assert float(b.norm()) > 0
    assert float((a - b).norm()) <= 1e-6 * float(b.norm())
    return int((ref_nn[..., 0] >= 0).sum())


def test_lookup_static_two_calls(lp):
    hits = [run_case(lp, *c, seed=20 + n) for n, c in enumerate(CASES)]
    assert all(h > 1000 for h in hits), hits


def test_lookup_static_rejects_bad_arguments(lp):
    prm = lp.GenParams(M=64, N=64, radius=float(np.sqrt(3.0)))
    img = torch.zeros((1, 8, 8, 3), device="cuda")
    cam = [lp.Camera((0.0, 0.0, 6.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.5)]
    with pytest.raises(lp.LumiPathError) as e:
        lp.lookup_static(torch.zeros((64, 64, 3), device="cuda"), prm, cam, 8, 8, 5, 7, img)
    assert e.value.code == -1
    with pytest.raises(lp.LumiPathError) as e:
        lp.lookup_static(torch.zeros((64, 64, 3), device="cuda"), prm, cam, 8, 8, 10, 0, img)
    assert e.value.code == -1
