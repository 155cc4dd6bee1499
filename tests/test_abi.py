"""The C ABI library loads, exports what include/lumipath.h declares, and its
host-side validation rejects bad arguments with the documented status codes
before any GPU work (runs without a GPU: none of these calls passes
validation, and size queries never touch the device)."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lumipath.h")

LF_OK, LF_E_ARG, LF_E_RANGE, LF_E_UNSUPPORTED, LF_E_WORKSPACE = 0, -1, -2, -3, -4
FAKE = C.c_void_p(0x10000)  # never dereferenced: validation fails first


@pytest.fixture(scope="module")
def lp():
    import paper_1903_03837_amd as lp
    if not os.path.exists(lp.library_path()):
        pytest.skip("liblumipath.so not built")
    return lp


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(lf_\w+)\s*\(", src, re.M)))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for f in ("lf_points", "lf_generate", "lf_lookup", "lf_generate_backward", "lf_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol(lp):
    L = lp.library()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert L.lf_version() == 1


def test_struct_layouts_match_header(lp):
    # sizes implied by the header's field order on LP64
    assert C.sizeof(lp._Volume) == 64
    assert C.sizeof(lp._Medium) == 16
    assert C.sizeof(lp._Light) == 76
    assert C.sizeof(lp._GenParams) == 112
    assert C.sizeof(lp._Camera) == 40


def scene(lp):
    vol = lp._Volume()
    vol.data = 0x10000
    vol.type, vol.nx, vol.ny, vol.nz, vol.brick = 0, 16, 16, 16, 0
    vol.vmin, vol.vmax = 0.0, 255.0
    vol.box_min[:] = [-1, -1, -1]
    vol.box_max[:] = [1, 1, 1]
    med = lp._Medium()
    med.lut, med.lut_size, med.density_scale = 0x20000, 256, 10.0
    light = lp._Light()
    light.kind = 0
    light.dir[:] = [0, 0, 1]
    light.radiance[:] = [1, 1, 1]
    prm = lp._GenParams()
    prm.M, prm.N, prm.radius, prm.spp, prm.max_bounces = 64, 64, math.sqrt(3), 4, 4
    return vol, med, light, prm


def call_generate(lp, vol, med, light, prm, dtype=0, out=FAKE, ws=None, ws_bytes=None):
    sz = C.c_size_t(0 if ws_bytes is None else ws_bytes)
    r = lp.library().lf_generate(C.byref(vol), C.byref(med), None, C.byref(light), C.byref(prm), dtype, out,
                                 ws, C.byref(sz), None)
    return r, sz.value


def err(lp):
    return lp.library().lf_last_error().decode()


def test_workspace_size_query(lp):
    vol, med, light, prm = scene(lp)
    r, sz = call_generate(lp, vol, med, light, prm)
    # majorant + counters, the spatial orders of 64 origins and 64 directions,
    # the point tables of both SF sets (16 B per point), then the halo-brick
    # copy of the 16^3 u8 volume: 5^3 bricks of 64 voxels (8000 B, rounded up
    # to 256 B)
    assert r == LF_OK and sz == 256 + 256 + 256 + 2048 + 8192


def test_workspace_size_with_majorant_grid(lp):
    vol, med, light, prm = scene(lp)
    prm.majorant_grid = 16
    r, sz = call_generate(lp, vol, med, light, prm)
    # the 16^3 cell majorants (16 KiB) sit between the spatial orders and the point tables
    assert r == LF_OK and sz == 256 + 256 + 256 + 16384 + 2048 + 8192
    prm.majorant = 2.0  # a fixed global majorant needs no grid
    assert call_generate(lp, vol, med, light, prm)[1] == 256 + 256 + 256 + 2048 + 8192


def test_majorant_grid_rejects(lp):
    vol, med, light, prm = scene(lp)
    L = lp.library()
    assert L.lf_majorant_grid(C.byref(vol), C.byref(med), C.byref(prm), FAKE, None) == LF_E_ARG  # grid 0
    prm.majorant_grid = 17
    assert L.lf_majorant_grid(C.byref(vol), C.byref(med), C.byref(prm), FAKE, None) == LF_E_ARG
    prm.majorant_grid = 4
    assert L.lf_majorant_grid(C.byref(vol), C.byref(med), C.byref(prm), None, None) == LF_E_ARG


@pytest.mark.parametrize("mutate,code,msg", [
    (lambda v, m, l, p: setattr(v, "data", None), LF_E_ARG, "data"),
    (lambda v, m, l, p: setattr(v, "type", 7), LF_E_ARG, "voxel type"),
    (lambda v, m, l, p: setattr(v, "nx", 1), LF_E_ARG, "dimensions"),
    (lambda v, m, l, p: (setattr(v, "brick", 8), setattr(v, "nx", 12)), LF_E_ARG, "multiples of 8"),
    (lambda v, m, l, p: setattr(v, "brick", 4), LF_E_UNSUPPORTED, "brick"),
    (lambda v, m, l, p: setattr(v, "vmax", -1.0), LF_E_ARG, "vmax"),
    (lambda v, m, l, p: setattr(v, "nx", 65536), LF_E_RANGE, "too large"),
    # 2048^3: its halo-brick copy (683^3 bricks of 64 voxels) passes 2^32 voxels
    (lambda v, m, l, p: (setattr(v, "nx", 2048), setattr(v, "ny", 2048), setattr(v, "nz", 2048)), LF_E_RANGE,
     "too large"),
    (lambda v, m, l, p: setattr(m, "lut_size", 1), LF_E_ARG, "lut_size"),
    (lambda v, m, l, p: setattr(m, "lut", 0x20004), LF_E_ARG, "aligned"),
    (lambda v, m, l, p: (setattr(v, "type", 2), setattr(v, "data", 0x10002)), LF_E_ARG, "aligned"),
    (lambda v, m, l, p: setattr(m, "density_scale", -1.0), LF_E_ARG, "density_scale"),
    (lambda v, m, l, p: setattr(l, "kind", 5), LF_E_ARG, "light kind"),
    (lambda v, m, l, p: l.dir.__setitem__(2, 2.0), LF_E_ARG, "unit vector"),
    (lambda v, m, l, p: setattr(p, "M", 0), LF_E_ARG, "M and N"),
    (lambda v, m, l, p: setattr(p, "N", 70000), LF_E_RANGE, "65535"),
    (lambda v, m, l, p: setattr(p, "spp", 0), LF_E_ARG, "spp"),
    (lambda v, m, l, p: setattr(p, "hg_g", 1.0), LF_E_ARG, "hg_g"),
    (lambda v, m, l, p: setattr(p, "radius", 0.0), LF_E_ARG, "radius"),
    (lambda v, m, l, p: setattr(p, "max_bounces", 0), LF_E_ARG, "max_bounces"),
    (lambda v, m, l, p: (setattr(p, "row_begin", 10), setattr(p, "row_end", 5)), LF_E_ARG, "row range"),
    (lambda v, m, l, p: setattr(p, "majorant_grid", 17), LF_E_ARG, "majorant_grid"),
    (lambda v, m, l, p: setattr(p, "majorant_grid", -1), LF_E_ARG, "majorant_grid"),
    (lambda v, m, l, p: setattr(p, "origin_rows", 65), LF_E_ARG, "origin_rows"),
    (lambda v, m, l, p: (setattr(p, "origin_rows", 32), setattr(p, "row_end", 40)), LF_E_ARG, "row range"),
])
def test_generate_rejects(lp, mutate, code, msg):
    vol, med, light, prm = scene(lp)
    mutate(vol, med, light, prm)
    r, _ = call_generate(lp, vol, med, light, prm)
    assert r == code
    assert msg in err(lp)


def test_sample_radiance_rejects(lp):
    vol, med, light, prm = scene(lp)
    prm.sample_radiance = 0x10002
    assert call_generate(lp, vol, med, light, prm)[0] == LF_E_ARG and "aligned" in err(lp)
    prm.sample_radiance = 0x10000
    prm.surface = 1
    assert call_generate(lp, vol, med, light, prm)[0] == LF_E_UNSUPPORTED


def test_generate_rejects_dtype_and_output(lp):
    vol, med, light, prm = scene(lp)
    assert call_generate(lp, vol, med, light, prm, dtype=3)[0] == LF_E_ARG
    assert call_generate(lp, vol, med, light, prm, out=None)[0] == LF_E_ARG


def test_generate_workspace_too_small(lp):
    vol, med, light, prm = scene(lp)
    r, _ = call_generate(lp, vol, med, light, prm, ws=FAKE, ws_bytes=16)
    assert r == LF_E_WORKSPACE and "workspace" in err(lp)


def test_backward_rejects_null_outputs(lp):
    vol, med, light, prm = scene(lp)
    sz = C.c_size_t(0)
    r = lp.library().lf_generate_backward(C.byref(vol), C.byref(med), C.byref(light), C.byref(prm), FAKE, None,
                                          FAKE, None, C.byref(sz), None)
    assert r == LF_E_ARG


def test_points_rejects(lp):
    L = lp.library()
    assert L.lf_points(0, FAKE, None, 0, 1, None, None, None) == LF_E_ARG
    assert L.lf_points(70000, FAKE, None, 0, 1, None, None, None) == LF_E_ARG
    assert L.lf_points(16, None, None, 0, 1, None, None, None) == LF_E_ARG
    assert L.lf_points(16, None, FAKE, 4, 10, FAKE, None, None) == LF_E_ARG
    assert L.lf_points(16, None, FAKE, 4, 5, None, None, None) == LF_E_ARG


def lookup(lp, cams, K=5, mode=0, W=8, H=8, lf=FAKE, img=FAKE, d_lf=None):
    _, _, _, prm = scene(lp)
    arr = lp._cams(cams)
    sz = C.c_size_t(1 << 20)
    return lp.library().lf_lookup(lf, 0, C.byref(prm), arr, len(cams), W, H, K, mode, img, d_lf, None, FAKE,
                                  C.byref(sz), None)


def test_lookup_rejects(lp):
    inside = lp.Camera((0.1, 0, 0), (1, 0, 0), (0, 0, 1), 0.5)
    assert lookup(lp, [inside]) == LF_E_ARG and "inside" in err(lp)
    parallel = lp.Camera((5, 0, 0), (0, 0, 0), (1, 0, 0), 0.5)
    assert lookup(lp, [parallel]) == LF_E_ARG and "parallel" in err(lp)
    badfov = lp.Camera((5, 0, 0), (0, 0, 0), (0, 0, 1), 3.5)
    assert lookup(lp, [badfov]) == LF_E_ARG
    ok = lp.Camera((5, 0, 0), (0, 0, 0), (0, 0, 1), 0.5)
    assert lookup(lp, [ok], K=0) == LF_E_ARG
    assert lookup(lp, [ok], K=10) == LF_E_ARG
    assert lookup(lp, [ok], mode=2) == LF_E_ARG
    assert lookup(lp, [ok], lf=None) == LF_E_ARG
    assert lookup(lp, [ok], mode=1, d_lf=None) == LF_E_ARG
    assert lookup(lp, [ok], W=0) == LF_E_ARG


def test_lookup_workspace_query(lp):
    _, _, _, prm = scene(lp)
    ok = lp.Camera((5, 0, 0), (0, 0, 0), (0, 0, 1), 0.5)
    arr = lp._cams([ok])
    sz = C.c_size_t(0)
    r = lp.library().lf_lookup(FAKE, 0, C.byref(prm), arr, 1, 8, 8, 5, 0, FAKE, None, None, None, C.byref(sz),
                               None)
    # the point tables of 64 + 64 SF points (16 B each), then the zone bases of both sets (768 B each)
    assert r == LF_OK and sz.value == 2 * 1024 + 2 * 768
    sz = C.c_size_t(100)
    r = lp.library().lf_lookup(FAKE, 0, C.byref(prm), arr, 1, 8, 8, 5, 0, FAKE, None, None, FAKE, C.byref(sz),
                               None)
    assert r == LF_E_WORKSPACE


def test_lookup_l2_rejects(lp):
    _, _, _, prm = scene(lp)
    ok = lp.Camera((5, 0, 0), (0, 0, 0), (0, 0, 1), 0.5)
    arr = lp._cams([ok])
    sz = C.c_size_t(1 << 20)
    L = lp.library()
    assert L.lf_lookup_l2(FAKE, 0, C.byref(prm), arr, 1, 8, 8, 5, None, FAKE, FAKE, FAKE, C.byref(sz), None) == LF_E_ARG
    assert "target" in err(lp)
    assert L.lf_lookup_l2(None, 0, C.byref(prm), arr, 1, 8, 8, 5, FAKE, FAKE, FAKE, FAKE, C.byref(sz), None) == LF_E_ARG
    assert L.lf_lookup_l2(FAKE, 0, C.byref(prm), arr, 1, 8, 8, 5, FAKE, FAKE, None, FAKE, C.byref(sz), None) == LF_E_ARG
    assert L.lf_lookup_l2(FAKE, 5, C.byref(prm), arr, 1, 8, 8, 5, FAKE, FAKE, FAKE, FAKE, C.byref(sz), None) == LF_E_ARG


def test_binding_refuses_to_run_without_library(tmp_path, monkeypatch):
    import paper_1903_03837_amd as lp
    monkeypatch.setattr(lp, "_lib", None)
    monkeypatch.setattr(lp, "_LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        lp.library()


def test_cw_ssim_workspace_and_rejects(lp):
    """lf_cw_ssim: workspace size query (no GPU call) and host-side rejects."""
    L = lp.library()
    a, b, out = C.c_void_p(0x10000), C.c_void_p(0x20000), C.c_void_p(0x30000)

    def query(W, H, rng=1.0, n=1, pa=a):
        sz = C.c_size_t(0)
        rc = L.lf_cw_ssim(pa, b, n, W, H, rng, out, None, C.byref(sz), None)
        return rc, sz.value

    def a256(x):
        return (x + 255) // 256 * 256

    for W, H in ((7, 7), (480, 270), (512, 512), (4096, 9)):
        rc, sz = query(W, H)
        assert rc == 0, lp.last_error() if hasattr(lp, "last_error") else rc
        gx, gy = (W - 6 + 15) // 16, (H - 6 + 15) // 16
        want = a256(8 * W) + a256(8 * H) + 3 * a256(48 * W * H) + a256(8 * gx * gy * 3 * 8)
        assert sz == want, (W, H, sz, want)
    assert query(6, 100)[0] == -1          # below the 7 x 7 window
    assert query(100, 6)[0] == -1
    assert query(4097, 100)[0] == -2       # DFT size limit
    assert query(100, 100, rng=-1.0)[0] == -1
    assert query(100, 100, rng=float("inf"))[0] == -1
    assert query(100, 100, n=0)[0] == -1
    assert query(100, 100, pa=None)[0] == -1
    assert query(100, 100, rng=0.0)[0] == 0  # K = 0 is allowed
