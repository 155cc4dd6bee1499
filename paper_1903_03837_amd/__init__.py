"""Python binding of liblumipath.so, the MI355X light-field library.

Argument marshalling only: every function below passes device pointers of
torch tensors, sizes and POD structs to the C ABI declared in
``include/lumipath.h`` and enqueues on ``torch.cuda.current_stream()``.  All
computation runs in the HIP kernels; if the shared library is missing this
module raises instead of computing anything another way.

Method: Fink et al., "LumiPath -- Towards Real-time Physically-based Rendering
on Embedded Devices" (arXiv 1903.03837), Sec. 2 (light field over two
spherical-Fibonacci point sets, its generation by path tracing, and image
synthesis by texel lookup), with a volumetric path tracer and two extensions
(FP16/BF16 storage, path-replay adjoint).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import torch

__all__ = [
    "LumiPathError", "Volume", "Medium", "Light", "GenParams", "Camera", "library", "library_path",
    "points", "generate", "generate_backward", "lookup", "majorant_grid", "render_views", "ssim", "lookup_adjoint", "LightFieldFn", "LookupFn",
    "device_scene", "DTYPES",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblumipath.so")

DTYPES = {"f32": 0, "f16": 1, "bf16": 2}
_TORCH_DTYPE = {0: torch.float32, 1: torch.float16, 2: torch.bfloat16}
VOX = {torch.uint8: 0, torch.int16: 1, torch.uint16: 1, torch.float32: 2}


class LumiPathError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lumipath error {code}: {msg}")
        self.code = code


# ----------------------------------------------------------------- C structs
class _Volume(C.Structure):
    _fields_ = [("data", C.c_void_p), ("type", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("brick", C.c_int32), ("vmin", C.c_float), ("vmax", C.c_float),
                ("box_min", C.c_float * 3), ("box_max", C.c_float * 3)]


class _Medium(C.Structure):
    _fields_ = [("lut", C.c_void_p), ("lut_size", C.c_int32), ("density_scale", C.c_float)]


class _Light(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dir", C.c_float * 3), ("corner", C.c_float * 3),
                ("e1", C.c_float * 3), ("e2", C.c_float * 3), ("radiance", C.c_float * 3),
                ("env", C.c_float * 3)]


class _GenParams(C.Structure):
    _fields_ = [("M", C.c_int32), ("N", C.c_int32), ("center", C.c_float * 3), ("radius", C.c_float),
                ("spp", C.c_int32), ("max_bounces", C.c_int32), ("hg_g", C.c_float), ("majorant", C.c_float),
                ("majorant_grid", C.c_int32),
                ("seed", C.c_uint64), ("jitter", C.c_int32), ("origin_rows", C.c_int32),
                ("row_begin", C.c_int64), ("row_end", C.c_int64), ("stats", C.c_void_p),
                ("surface", C.c_int32), ("iso", C.c_float), ("sample_radiance", C.c_void_p),
                ("waves_per_simd", C.c_int32)]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3), ("vfov", C.c_float)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def library():
    """Load liblumipath.so (built in-tree by build.py); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built: run paper_1903_03837_amd/build.py "
                               "(or __graft_entry__.build()) first")
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        L.lf_last_error.restype = C.c_char_p
        L.lf_version.restype = C.c_int
        L.lf_points.argtypes = [C.c_int32, P, P, C.c_int64, C.c_int32, P, P, P]
        L.lf_generate.argtypes = [P, P, P, P, P, C.c_int32, P, P, C.POINTER(C.c_size_t), P]
        L.lf_generate_backward.argtypes = [P, P, P, P, P, P, P, P, C.POINTER(C.c_size_t), P]
        L.lf_lookup.argtypes = [P, C.c_int32, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                P, P, P, P, C.POINTER(C.c_size_t), P]
        L.lf_lookup_static.argtypes = [P, C.c_int32, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                       C.c_int32, P, P, P, P]
        L.lf_lookup_l2.argtypes = [P, C.c_int32, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, P, P,
                                   C.POINTER(C.c_size_t), P]
        L.lf_majorant_grid.argtypes = [P, P, P, P, P]
        L.lf_render_views.argtypes = [P, P, P, P, P, C.c_int32, C.c_int32, C.c_int32, P, P,
                                      C.POINTER(C.c_size_t), P]
        L.lf_ssim.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, C.POINTER(C.c_size_t), P]
        L.lf_cw_ssim.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, C.POINTER(C.c_size_t), P]
        for f in (L.lf_points, L.lf_generate, L.lf_generate_backward, L.lf_lookup, L.lf_lookup_static, L.lf_lookup_l2,
                  L.lf_majorant_grid, L.lf_render_views, L.lf_ssim, L.lf_cw_ssim):
            f.restype = C.c_int
        _lib = L
    return _lib


def _check(code: int):
    if code != 0:
        raise LumiPathError(code, library().lf_last_error().decode())


def _need(t: torch.Tensor, numel: int, dtypes, name: str):
    """The C ABI takes plain device pointers: check here that a buffer holds
    what the call will read or write."""
    if not isinstance(dtypes, tuple):
        dtypes = (dtypes,)
    if t.dtype not in dtypes:
        raise ValueError(f"{name}: dtype {t.dtype} not in {dtypes}")
    if t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, {numel} needed")


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


# ----------------------------------------------------------------- records
@dataclass
class Volume:
    data: torch.Tensor                       # device, 1-D in storage order
    dims: Tuple[int, int, int]
    vmin: float
    vmax: float
    brick: int = 0
    box_min: Tuple[float, float, float] = (-1.0, -1.0, -1.0)
    box_max: Tuple[float, float, float] = (1.0, 1.0, 1.0)

    def c(self) -> _Volume:
        s = _Volume()
        s.data = self.data.data_ptr()
        s.type = VOX[self.data.dtype]
        s.nx, s.ny, s.nz = self.dims
        s.brick = self.brick
        s.vmin, s.vmax = self.vmin, self.vmax
        s.box_min[:] = list(self.box_min)
        s.box_max[:] = list(self.box_max)
        return s


@dataclass
class Medium:
    lut: torch.Tensor                        # device float32 [L, 4]
    scale: float

    def c(self) -> _Medium:
        if self.lut.dtype != torch.float32 or self.lut.dim() != 2 or self.lut.shape[1] != 4:
            raise ValueError("lut must be float32 [L, 4]")
        s = _Medium()
        s.lut = _ptr(self.lut).value
        s.lut_size = self.lut.shape[0]
        s.density_scale = float(self.scale)
        return s


@dataclass
class Light:
    kind: int                                # 0 directional, 1 area
    dir: Sequence[float] = (0.0, 0.0, 1.0)
    corner: Sequence[float] = (0.0, 0.0, 0.0)
    e1: Sequence[float] = (0.0, 0.0, 0.0)
    e2: Sequence[float] = (0.0, 0.0, 0.0)
    radiance: Sequence[float] = (1.0, 1.0, 1.0)
    env: Sequence[float] = (0.0, 0.0, 0.0)

    def c(self) -> _Light:
        s = _Light()
        s.kind = self.kind
        for f in ("dir", "corner", "e1", "e2", "radiance", "env"):
            getattr(s, f)[:] = [float(x) for x in getattr(self, f)]
        return s


@dataclass
class GenParams:
    M: int
    N: int
    center: Sequence[float] = (0.0, 0.0, 0.0)
    radius: float = math.sqrt(3.0)
    spp: int = 16
    max_bounces: int = 4
    g: float = 0.0
    majorant: float = 0.0
    seed: int = 0
    jitter: int = 1
    row_begin: int = 0
    row_end: int = 0
    origin_rows: int = 0                     # 0: all M origins; M // 2: upper hemisphere
    grid: int = 0                            # majorant grid cells per axis (0: one global majorant)
    surface: int = 0                         # 1: isosurface variant at raw value iso
    iso: float = 0.0
    waves_per_simd: int = 0                  # forward tracer's register budget: 0 (library's choice), 3 or 4

    @property
    def rows(self) -> int:
        return self.origin_rows if self.origin_rows > 0 else self.M

    def c(self, stats: Optional[torch.Tensor] = None, sample_radiance: Optional[torch.Tensor] = None) -> _GenParams:
        s = _GenParams()
        s.M, s.N = self.M, self.N
        s.center[:] = [float(x) for x in self.center]
        s.radius = self.radius
        s.spp, s.max_bounces = self.spp, self.max_bounces
        s.hg_g, s.majorant = self.g, self.majorant
        s.majorant_grid = self.grid
        s.surface, s.iso = self.surface, self.iso
        s.waves_per_simd = self.waves_per_simd
        s.seed = self.seed
        s.jitter = self.jitter
        s.origin_rows = self.origin_rows
        s.row_begin, s.row_end = self.row_begin, self.row_end
        if stats is not None:
            _need(stats, 5, torch.int64, "stats")
        s.stats = _ptr(stats).value if stats is not None else None
        if sample_radiance is not None:
            _need(sample_radiance, self.rows * self.N * self.spp * 3, torch.float32, "sample_radiance")
        s.sample_radiance = _ptr(sample_radiance).value if sample_radiance is not None else None
        return s


@dataclass
class Camera:
    eye: Sequence[float]
    target: Sequence[float]
    up: Sequence[float]
    vfov: float


def _cams(cams: Sequence[Camera]):
    arr = (_Camera * len(cams))()
    for a, c in zip(arr, cams):
        a.eye[:] = [float(x) for x in c.eye]
        a.target[:] = [float(x) for x in c.target]
        a.up[:] = [float(x) for x in c.up]
        a.vfov = float(c.vfov)
    return arr


def device_scene(scene, device="cuda"):
    """Copy a host scene description (any object with volume / medium /
    light / params / cams attributes holding numpy arrays, e.g. an
    ``lfsynth.Scene``) to the device records above."""
    import numpy as np
    v = scene.volume
    data = torch.from_numpy(np.ascontiguousarray(v.data))
    if data.dtype == torch.uint16:
        data = data.view(torch.int16)
    vol = Volume(data.to(device), tuple(v.dims), float(v.vmin), float(v.vmax), int(v.brick),
                 tuple(v.box_min), tuple(v.box_max))
    med = Medium(torch.from_numpy(np.ascontiguousarray(scene.medium.lut, dtype=np.float32)).to(device),
                 float(scene.medium.scale))
    l = scene.light
    light = Light(int(l.kind), l.dir, l.corner, l.e1, l.e2, l.radiance, l.env)
    p = scene.params
    prm = GenParams(int(p.M), int(p.N), tuple(p.center), float(p.radius), int(p.spp), int(p.max_bounces),
                    float(p.g), float(p.majorant), int(p.seed), int(p.jitter),
                    origin_rows=int(getattr(p, "origin_rows", 0)), grid=int(getattr(p, "grid", 0)),
                    surface=int(getattr(p, "surface", 0)), iso=float(getattr(p, "iso", 0.0)))
    cams = [Camera(c.eye, c.target, c.up, c.vfov) for c in getattr(scene, "cams", [])]
    return vol, med, light, prm, cams


# ----------------------------------------------------------------- functions
def points(n: int, query: Optional[torch.Tensor] = None, K: int = 1, want_xyz: bool = True,
           device="cuda"):
    """lf_points: (xyz [n,3] or None, idx [nq,K] or None, w [nq,K] or None)."""
    xyz = torch.empty((n, 3), dtype=torch.float32, device=device) if want_xyz else None
    idx = w = None
    nq = 0
    if query is not None:
        query = query.contiguous()
        nq = query.shape[0]
        idx = torch.empty((nq, K), dtype=torch.int32, device=query.device)
        w = torch.empty((nq, K), dtype=torch.float32, device=query.device)
    _check(library().lf_points(n, _ptr(xyz), _ptr(query), nq, K, _ptr(idx), _ptr(w), _stream()))
    return xyz, idx, w


def _workspace(fn, *args) -> torch.Tensor:
    sz = C.c_size_t(0)
    _check(fn(*args, None, C.byref(sz), None))
    return torch.empty(max(int(sz.value), 16), dtype=torch.uint8, device="cuda"), sz


def generate(vol: Volume, med: Medium, light: Light, prm: GenParams, dtype: str = "f32",
             sample: Optional[Medium] = None, out: Optional[torch.Tensor] = None,
             stats: Optional[torch.Tensor] = None, sample_radiance: Optional[torch.Tensor] = None) -> torch.Tensor:
    """lf_generate: light field [rows, N, 3] of `dtype` ('f32', 'f16', 'bf16'),
    rows = prm.origin_rows or M.  sample_radiance: None or float32
    [rows, N, spp, 3] that receives every sample's radiance (for
    generate_backward)."""
    dt = DTYPES[dtype]
    if out is None:
        out = torch.empty((prm.rows, prm.N, 3), dtype=_TORCH_DTYPE[dt], device=vol.data.device)
    _need(out, prm.rows * prm.N * 3, _TORCH_DTYPE[dt], "out")
    L = library()
    v, m, l, p = vol.c(), med.c(), light.c(), prm.c(stats, sample_radiance)
    s = sample.c() if sample is not None else None
    args = [C.byref(v), C.byref(m), C.byref(s) if s is not None else None, C.byref(l), C.byref(p), dt,
            _ptr(out)]
    ws, sz = _workspace(L.lf_generate, *args)
    _check(L.lf_generate(*args, _ptr(ws), C.byref(sz), _stream()))
    return out


def render_views(vol: Volume, med: Medium, light: Light, prm: GenParams, cams: Sequence[Camera], width: int,
                 height: int, img: Optional[torch.Tensor] = None) -> torch.Tensor:
    """lf_render_views: ground-truth images [V, H, W, 3] (float32), prm.spp
    path samples per pixel along the pinhole rays."""
    V = len(cams)
    if img is None:
        img = torch.empty((V, height, width, 3), dtype=torch.float32, device=vol.data.device)
    _need(img, V * height * width * 3, torch.float32, "img")
    L = library()
    v, m, l, p = vol.c(), med.c(), light.c(), prm.c()
    cs = _cams(cams)
    args = [C.byref(v), C.byref(m), C.byref(l), C.byref(p), cs, V, width, height, _ptr(img)]
    ws, sz = _workspace(L.lf_render_views, *args)
    _check(L.lf_render_views(*args, _ptr(ws), C.byref(sz), _stream()))
    return img


def ssim(a: torch.Tensor, b: torch.Tensor, data_range: float = 1.0) -> torch.Tensor:
    """lf_ssim: mean SSIM [n] (float64) of image pairs [n, H, W, 3] (float32)."""
    if a.shape != b.shape or a.dim() != 4 or a.shape[-1] != 3:
        raise ValueError("a and b must both be [n, H, W, 3]")
    a = a.contiguous().float()
    b = b.contiguous().float()
    n, H, W, _ = a.shape
    out = torch.empty(n, dtype=torch.float64, device=a.device)
    L = library()
    args = [_ptr(a), _ptr(b), n, W, H, float(data_range), _ptr(out)]
    ws, sz = _workspace(L.lf_ssim, *args)
    _check(L.lf_ssim(*args, _ptr(ws), C.byref(sz), _stream()))
    return out


def cw_ssim(a: torch.Tensor, b: torch.Tensor, data_range: float = 1.0) -> torch.Tensor:
    """lf_cw_ssim: mean CW-SSIM [n] (float64) of image pairs [n, H, W, 3] (float32)."""
    if a.shape != b.shape or a.dim() != 4 or a.shape[-1] != 3:
        raise ValueError("a and b must both be [n, H, W, 3]")
    a = a.contiguous().float()
    b = b.contiguous().float()
    n, H, W, _ = a.shape
    out = torch.empty(n, dtype=torch.float64, device=a.device)
    L = library()
    args = [_ptr(a), _ptr(b), n, W, H, float(data_range), _ptr(out)]
    ws, sz = _workspace(L.lf_cw_ssim, *args)
    _check(L.lf_cw_ssim(*args, _ptr(ws), C.byref(sz), _stream()))
    return out


def majorant_grid(vol: Volume, med: Medium, prm: GenParams) -> torch.Tensor:
    """lf_majorant_grid: cell majorants [G, G, G] (z, y, x) for G = prm.grid."""
    G = prm.grid
    if G < 1:
        raise ValueError("prm.grid must be >= 1")
    out = torch.empty((G, G, G), dtype=torch.float32, device=med.lut.device)
    v, m, p = vol.c(), med.c(), prm.c()
    _check(library().lf_majorant_grid(C.byref(v), C.byref(m), C.byref(p), _ptr(out), _stream()))
    return out


def generate_backward(vol: Volume, med: Medium, light: Light, prm: GenParams, d_lf: torch.Tensor,
                      sample_radiance: Optional[torch.Tensor] = None):
    """lf_generate_backward: (d_lut [L,4], d_scale [1]) for d(loss)/d(Lhat).
    sample_radiance: None, or the per-sample radiance that generate() kept
    with the same parameters and medium (the first replay pass is skipped)."""
    d_lf = d_lf.contiguous().float()
    _need(d_lf, prm.rows * prm.N * 3, torch.float32, "d_lf")
    d_lut = torch.empty_like(med.lut)
    d_scale = torch.empty(1, dtype=torch.float32, device=med.lut.device)
    L = library()
    v, m, l, p = vol.c(), med.c(), light.c(), prm.c(sample_radiance=sample_radiance)
    args = [C.byref(v), C.byref(m), C.byref(l), C.byref(p), _ptr(d_lf), _ptr(d_lut), _ptr(d_scale)]
    ws, sz = _workspace(L.lf_generate_backward, *args)
    _check(L.lf_generate_backward(*args, _ptr(ws), C.byref(sz), _stream()))
    return d_lut, d_scale


def lookup(lf: torch.Tensor, prm: GenParams, cams: Sequence[Camera], width: int, height: int, K: int = 5,
           with_nn: bool = False, img: Optional[torch.Tensor] = None):
    """lf_lookup forward: images [V, H, W, 3] (and nearest (i, j) [V, H, W, 2])."""
    dt = {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2}[lf.dtype]
    V = len(cams)
    _need(lf, prm.rows * prm.N * 3, lf.dtype, "lf")
    if img is None:
        img = torch.empty((V, height, width, 3), dtype=torch.float32, device=lf.device)
    _need(img, V * height * width * 3, torch.float32, "img")
    nn = torch.empty((V, height, width, 2), dtype=torch.int32, device=lf.device) if with_nn else None
    p = prm.c()
    cs = _cams(cams)
    args = [_ptr(lf), dt, C.byref(p), cs, V, width, height, K, 0, _ptr(img), None, _ptr(nn)]
    ws, sz = _workspace(library().lf_lookup, *args)
    _check(library().lf_lookup(*args, _ptr(ws), C.byref(sz), _stream()))
    return (img, nn) if with_nn else img


def lookup_static(lf: Optional[torch.Tensor], prm: GenParams, cams: Sequence[Camera], width: int, height: int,
                  K: int, mode: int, img: torch.Tensor, d_lf: Optional[torch.Tensor] = None,
                  nn: Optional[torch.Tensor] = None) -> None:
    """lf_lookup_static: lf_lookup with the library's fixed scratch (no
    workspace).  Every buffer is the caller's: mode 0 writes img (and nn),
    mode 1 adds the transpose of img to d_lf."""
    V = len(cams)
    dt = 0 if lf is None else {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2}[lf.dtype]
    if lf is not None:
        _need(lf, prm.rows * prm.N * 3, lf.dtype, "lf")
    _need(img, V * height * width * 3, torch.float32, "img")
    if d_lf is not None:
        _need(d_lf, prm.rows * prm.N * 3, torch.float32, "d_lf")
    if nn is not None:
        _need(nn, V * height * width * 2, torch.int32, "nn")
    p = prm.c()
    _check(library().lf_lookup_static(_ptr(lf), dt, C.byref(p), _cams(cams), V, width, height, K, mode,
                                      _ptr(img), _ptr(d_lf), _ptr(nn), _stream()))


def lookup_adjoint(dimg: torch.Tensor, prm: GenParams, cams: Sequence[Camera], K: int = 5,
                   d_lf: Optional[torch.Tensor] = None) -> torch.Tensor:
    """lf_lookup adjoint: d_lf [rows, N, 3] (float32) += transpose applied to dimg."""
    dimg = dimg.contiguous().float()
    V, H, W, _ = dimg.shape
    if d_lf is None:
        d_lf = torch.zeros((prm.rows, prm.N, 3), dtype=torch.float32, device=dimg.device)
    _need(d_lf, prm.rows * prm.N * 3, torch.float32, "d_lf")
    p = prm.c()
    cs = _cams(cams)
    args = [None, 0, C.byref(p), cs, V, W, H, K, 1, _ptr(dimg), _ptr(d_lf), None]
    ws, sz = _workspace(library().lf_lookup, *args)
    _check(library().lf_lookup(*args, _ptr(ws), C.byref(sz), _stream()))
    return d_lf


def lookup_l2(lf: torch.Tensor, prm: GenParams, cams: Sequence[Camera], target: torch.Tensor, K: int = 5,
              img: Optional[torch.Tensor] = None, d_lf: Optional[torch.Tensor] = None):
    """lf_lookup_l2: (img [V, H, W, 3], d_lf [rows, N, 3]); img = lookup(lf),
    d_lf += lookup transpose of (img - target)."""
    dt = {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2}[lf.dtype]
    target = target.contiguous().float()
    V, H, W, _ = target.shape
    _need(lf, prm.rows * prm.N * 3, lf.dtype, "lf")
    if img is None:
        img = torch.empty_like(target)
    _need(img, V * H * W * 3, torch.float32, "img")
    if d_lf is None:
        d_lf = torch.zeros((prm.rows, prm.N, 3), dtype=torch.float32, device=lf.device)
    _need(d_lf, prm.rows * prm.N * 3, torch.float32, "d_lf")
    p = prm.c()
    cs = _cams(cams)
    args = [_ptr(lf), dt, C.byref(p), cs, V, W, H, K, _ptr(target), _ptr(img), _ptr(d_lf)]
    ws, sz = _workspace(library().lf_lookup_l2, *args)
    _check(library().lf_lookup_l2(*args, _ptr(ws), C.byref(sz), _stream()))
    return img, d_lf


# ----------------------------------------------------------------- autograd
class LightFieldFn(torch.autograd.Function):
    """Lhat = generate(LUT, density scale); backward by path replay
    (lf_generate_backward).  `scale` is a 0-d float tensor on the CPU.  With
    keep_samples the forward keeps every sample's radiance (rows x N x spp x
    12 bytes) so that the backward traces each sample once instead of twice."""

    @staticmethod
    def forward(ctx, lut, scale, vol, light, prm, keep_samples=False):
        med = Medium(lut.detach().contiguous(), float(scale))
        ctx.vol, ctx.light, ctx.prm = vol, light, prm
        ctx.save_for_backward(lut, scale)
        ctx.srad = None
        if keep_samples:
            ctx.srad = torch.empty((prm.rows, prm.N, prm.spp, 3), dtype=torch.float32, device=lut.device)
        return generate(vol, med, light, prm, sample_radiance=ctx.srad)

    @staticmethod
    def backward(ctx, g):
        lut, scale = ctx.saved_tensors
        d_lut, d_scale = generate_backward(ctx.vol, Medium(lut.detach().contiguous(), float(scale)), ctx.light,
                                           ctx.prm, g, sample_radiance=ctx.srad)
        ctx.srad = None
        return d_lut, d_scale.to(scale.device).reshape(scale.shape), None, None, None, None


class LookupFn(torch.autograd.Function):
    """Views = lookup(Lhat); backward scatters through the same weights."""

    @staticmethod
    def forward(ctx, lf, prm, cams, width, height, K):
        ctx.prm, ctx.cams, ctx.K = prm, cams, K
        return lookup(lf, prm, cams, width, height, K)

    @staticmethod
    def backward(ctx, g):
        return lookup_adjoint(g, ctx.prm, ctx.cams, ctx.K), None, None, None, None, None
