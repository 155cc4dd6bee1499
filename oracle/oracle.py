"""ctypes front end of the FP64 CPU oracle (``liblforacle.so``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the GPU library never does.  Inputs are
plain numpy arrays and objects carrying the attributes of the ``lfsynth``
scene records (volume, medium, light, params, cameras); nothing here imports
the GPU package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblforacle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O2, no fast-math)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
               "-o", _SO + ".tmp", os.path.join(_HERE, "lforacle.c"), "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Volume(C.Structure):
    _fields_ = [("data", C.c_void_p), ("type", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("brick", C.c_int32), ("vmin", C.c_double), ("vmax", C.c_double),
                ("box_min", C.c_double * 3), ("box_max", C.c_double * 3)]


class _Medium(C.Structure):
    _fields_ = [("lut", C.c_void_p), ("lut_size", C.c_int32), ("scale", C.c_double)]


class _Light(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dir", C.c_double * 3), ("corner", C.c_double * 3),
                ("e1", C.c_double * 3), ("e2", C.c_double * 3), ("radiance", C.c_double * 3),
                ("env", C.c_double * 3)]


class _Params(C.Structure):
    _fields_ = [("M", C.c_int64), ("N", C.c_int64), ("center", C.c_double * 3), ("radius", C.c_double),
                ("spp", C.c_int32), ("max_bounces", C.c_int32), ("g", C.c_double),
                ("majorant", C.c_double), ("seed", C.c_uint64), ("jitter", C.c_int32),
                ("grid", C.c_int32), ("surface", C.c_int32), ("iso", C.c_double), ("origin_rows", C.c_int64)]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("vfov", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        L.orc_sf_point.argtypes = [C.c_int64, C.c_int64, P]
        L.orc_sf_points.argtypes = [C.c_int64, P]
        L.orc_nearest.argtypes = [C.c_int64, P, P, P]
        L.orc_nearest.restype = C.c_int64
        L.orc_zone.argtypes = [C.c_int64, C.c_double, P]
        L.orc_zone.restype = C.c_int32
        L.orc_fib.argtypes = [C.c_int32]
        L.orc_fib.restype = C.c_int64
        L.orc_neighbors.argtypes = [C.c_int64, P, C.c_int32, P, P, P, P]
        L.orc_neighbors.restype = C.c_int32
        L.orc_neighbors_batch.argtypes = [C.c_int64, P, C.c_int64, C.c_int32, P, P, P, P, P, C.c_int32]
        L.orc_philox.argtypes = [P, P, P]
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_hg_phase.argtypes = [C.c_double, C.c_double]
        L.orc_hg_phase.restype = C.c_double
        L.orc_hg_sample_mu.argtypes = [C.c_double, C.c_double]
        L.orc_hg_sample_mu.restype = C.c_double
        L.orc_frame.argtypes = [P, P, P]
        L.orc_majorant.argtypes = [P, P]
        L.orc_majorant.restype = C.c_double
        L.orc_majorant_grid.argtypes = [P, P, P, P]
        L.orc_sigma_at.argtypes = [P, P, P, C.c_int64, P]
        L.orc_generate.argtypes = [P, P, P, P, P, P, C.c_int64, P, C.c_int32, P]
        L.orc_gradient.argtypes = [P, P, P, P, P, C.c_int64, P, P, P, C.c_int32]
        L.orc_lookup.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int32, P, C.c_int64, P, P, P, C.c_int32]
        L.orc_lookup_adjoint.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, P, C.c_int64, P, P]
        L.orc_render.argtypes = [P, P, P, P, P, C.c_int32, C.c_int32, P, C.c_int64, P, C.c_int32]
        L.orc_ssim.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32, C.c_double, P]
        L.orc_surface_hit.argtypes = [P, P, P, P, C.c_double, C.c_double, P]
        L.orc_surface_hit.restype = C.c_int32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


# ------------------------------------------------------------------ marshalling
def _vol(v, keep):
    data = np.ascontiguousarray(v.data)
    keep.append(data)
    s = _Volume()
    s.data = data.ctypes.data
    s.type = v.vtype
    s.nx, s.ny, s.nz = v.dims
    s.brick = v.brick
    s.vmin, s.vmax = v.vmin, v.vmax
    s.box_min[:] = list(v.box_min)
    s.box_max[:] = list(v.box_max)
    return s


def _med(m, keep):
    lut = np.ascontiguousarray(m.lut, dtype=np.float32)
    keep.append(lut)
    s = _Medium()
    s.lut = lut.ctypes.data
    s.lut_size = lut.shape[0]
    s.scale = float(m.scale)
    return s


def _light(l):
    s = _Light()
    s.kind = l.kind
    s.dir[:] = list(l.dir)
    s.corner[:] = list(l.corner)
    s.e1[:] = list(l.e1)
    s.e2[:] = list(l.e2)
    s.radiance[:] = list(l.radiance)
    s.env[:] = list(l.env)
    return s


def _params(p):
    s = _Params()
    s.M, s.N = p.M, p.N
    s.center[:] = list(p.center)
    s.radius = p.radius
    s.spp, s.max_bounces = p.spp, p.max_bounces
    s.g = p.g
    s.majorant = p.majorant
    s.seed = p.seed
    s.jitter = p.jitter
    s.grid = getattr(p, "grid", 0)
    s.surface = getattr(p, "surface", 0)
    s.iso = getattr(p, "iso", 0.0)
    s.origin_rows = getattr(p, "origin_rows", 0)
    return s


def stored_rows(p) -> int:
    """Rows of origins the light field stores (origin_rows, 0 meaning M)."""
    r = getattr(p, "origin_rows", 0)
    return r if r > 0 else p.M


def _cams(cams):
    arr = (_Camera * len(cams))()
    for a, c in zip(arr, cams):
        a.eye[:] = list(c.eye)
        a.target[:] = list(c.target)
        a.up[:] = list(c.up)
        a.vfov = c.vfov
    return arr


# ------------------------------------------------------------------ functions
def sf_points(n: int) -> np.ndarray:
    out = np.empty((n, 3))
    lib().orc_sf_points(n, _ptr(out))
    return out


def nearest(n: int, q) -> tuple:
    q = np.ascontiguousarray(q, dtype=np.float64)
    b, s = C.c_double(), C.c_double()
    i = lib().orc_nearest(n, _ptr(q), C.byref(b), C.byref(s))
    return i, b.value, s.value


def zone(n: int, qz: float) -> tuple:
    m = C.c_double()
    k = lib().orc_zone(n, qz, C.byref(m))
    return k, m.value


def fib(k: int) -> int:
    return lib().orc_fib(k)


def neighbors(n: int, q, K: int):
    """(indices, weights, squared distances, margins) of the K-neighbour query."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    idx = np.zeros(9, np.int64)
    w = np.zeros(9)
    d2 = np.zeros(9)
    m = np.zeros(3)
    cnt = lib().orc_neighbors(n, _ptr(q), K, _ptr(idx), _ptr(w), _ptr(d2), _ptr(m))
    return idx[:cnt], w[:cnt], d2[:cnt], m


def neighbors_batch(n: int, q, K: int, nthreads=None):
    """Batched K-neighbour query: idx [nq,K] (-1 past the count), w, d2
    [nq,K], margins [nq,3], count [nq]."""
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
    nq = q.shape[0]
    idx = np.zeros((nq, K), np.int64)
    w = np.zeros((nq, K))
    d2 = np.zeros((nq, K))
    m = np.zeros((nq, 3))
    cnt = np.zeros(nq, np.int32)
    lib().orc_neighbors_batch(n, _ptr(q), nq, K, _ptr(idx), _ptr(w), _ptr(d2), _ptr(m), _ptr(cnt),
                              nthreads or default_threads())
    return idx, w, d2, m, cnt


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(x: int) -> float:
    return lib().orc_uniform(x)


def majorant(medium, params) -> float:
    keep = []
    m = _med(medium, keep)
    p = _params(params)
    return lib().orc_majorant(C.byref(m), C.byref(p))


def majorant_grid(volume, medium, params) -> np.ndarray:
    """Cell majorants [G, G, G] (z, y, x) of the majorant grid, G = params.grid."""
    keep = []
    v = _vol(volume, keep)
    m = _med(medium, keep)
    p = _params(params)
    G = int(params.grid)
    if not 1 <= G <= 64:
        raise ValueError("grid must be in [1, 64]")
    out = np.zeros(G * G * G)
    lib().orc_majorant_grid(C.byref(v), C.byref(m), C.byref(p), _ptr(out))
    return out.reshape(G, G, G)


def sigma_at(volume, medium, pts) -> np.ndarray:
    """sigma_t of `medium` at world points pts [n, 3]."""
    keep = []
    v = _vol(volume, keep)
    m = _med(medium, keep)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(len(pts))
    lib().orc_sigma_at(C.byref(v), C.byref(m), _ptr(pts), len(pts), _ptr(out))
    return out


def generate(scene, rays, sample_medium=None, nthreads=None, stats=False):
    """Mean radiance [len(rays), 3] (float64) of the listed rays k = i*N + j."""
    keep = []
    rays = np.ascontiguousarray(rays, dtype=np.int64)
    out = np.zeros((len(rays), 3))
    v = _vol(scene.volume, keep)
    e = _med(scene.medium, keep)
    s = _med(sample_medium, keep) if sample_medium is not None else None
    l = _light(scene.light)
    p = _params(scene.params)
    st = np.zeros(4)
    lib().orc_generate(C.byref(v), C.byref(e), C.byref(s) if s is not None else None, C.byref(l),
                       C.byref(p), _ptr(rays), len(rays), _ptr(out), nthreads or default_threads(),
                       _ptr(st))
    return (out, st) if stats else out


def gradient(scene, rays, adj, nthreads=None):
    """(d_lut [L,4], d_scale) of sum_r adj[r] . Lhat(rays[r])."""
    keep = []
    rays = np.ascontiguousarray(rays, dtype=np.int64)
    adj = np.ascontiguousarray(adj, dtype=np.float64).reshape(len(rays), 3)
    v = _vol(scene.volume, keep)
    m = _med(scene.medium, keep)
    l = _light(scene.light)
    p = _params(scene.params)
    d_lut = np.zeros((m.lut_size, 4))
    d_scale = np.zeros(1)
    lib().orc_gradient(C.byref(v), C.byref(m), C.byref(l), C.byref(p), _ptr(rays), len(rays),
                       _ptr(adj), _ptr(d_lut), _ptr(d_scale), nthreads or default_threads())
    return d_lut, float(d_scale[0])


def lookup(lf, params, cams, width, height, K, pix, nthreads=None):
    """RGB [npx,3], nearest (i,j) [npx,2], margins [npx,4] of the listed pixels
    pix = [(view, x, y), ...] over the FP32 light field lf [rows*N*3]."""
    lf = np.ascontiguousarray(lf, dtype=np.float32).reshape(-1)
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    n = pix.shape[0]
    rgb = np.zeros((n, 3))
    nn = np.zeros((n, 2), np.int64)
    mg = np.zeros((n, 4))
    p = _params(params)
    cs = _cams(cams)
    lib().orc_lookup(_ptr(lf), C.byref(p), cs, width, height, K, _ptr(pix), n, _ptr(rgb), _ptr(nn),
                     _ptr(mg), nthreads or default_threads())
    return rgb, nn, mg


def lookup_adjoint(params, cams, width, height, K, pix, dimg) -> np.ndarray:
    """FP64 d_lf [rows*N*3] = transpose of lookup applied to dimg [npx,3]."""
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    dimg = np.ascontiguousarray(dimg, dtype=np.float64).reshape(-1, 3)
    p = _params(params)
    cs = _cams(cams)
    d = np.zeros(stored_rows(params) * params.N * 3)
    lib().orc_lookup_adjoint(C.byref(p), cs, width, height, K, _ptr(pix), pix.shape[0], _ptr(dimg), _ptr(d))
    return d


def render(scene, cams, width, height, pix, nthreads=None) -> np.ndarray:
    """Ground-truth RGB [npx, 3] of the listed pixels pix = [(view, x, y), ...]:
    mean over spp path samples along each pinhole ray."""
    keep = []
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    out = np.zeros((pix.shape[0], 3))
    v = _vol(scene.volume, keep)
    m = _med(scene.medium, keep)
    l = _light(scene.light)
    p = _params(scene.params)
    cs = _cams(cams)
    lib().orc_render(C.byref(v), C.byref(m), C.byref(l), C.byref(p), cs, width, height, _ptr(pix), pix.shape[0],
                     _ptr(out), nthreads or default_threads())
    return out


def surface_hit(volume, params, x, d, t0, t1):
    """First isosurface crossing along x + t d in [t0, t1): t, or None."""
    keep = []
    v = _vol(volume, keep)
    p = _params(params)
    x = np.ascontiguousarray(x, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    th = C.c_double()
    ok = lib().orc_surface_hit(C.byref(v), C.byref(p), _ptr(x), _ptr(d), t0, t1, C.byref(th))
    return th.value if ok else None


def ssim(a, b, data_range=1.0) -> np.ndarray:
    """Mean SSIM [n] of float32 image pairs [n, H, W, 3]."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    n, H, W, _ = a.shape
    out = np.zeros(n)
    lib().orc_ssim(_ptr(a), _ptr(b), n, W, H, data_range, _ptr(out))
    return out


def all_pixels(nviews: int, width: int, height: int) -> np.ndarray:
    v, y, x = np.meshgrid(np.arange(nviews), np.arange(height), np.arange(width), indexing="ij")
    return np.stack([v.ravel(), x.ravel(), y.ravel()], -1).astype(np.int32)
