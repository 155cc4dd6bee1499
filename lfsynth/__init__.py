"""Seeded synthetic inputs for the light-field path.

The paper's scenes are CT-derived surfaces and a skull model that are not
available; these volumes stand in for them (Gaussian-blob densities and a
nested-ellipsoid CT-like phantom).  This module only *makes inputs*: voxel
arrays, transfer-function tables, lights, cameras and run parameters.  It
holds none of the method's arithmetic, so that the CPU oracle and the GPU
library can both be fed from it without sharing any code.

Every array is produced from ``numpy.random.default_rng(seed)`` with the
fixed seeds below, so the same call always returns the same bytes.

Seeds per workload c (1..5): volume 1000+c, transfer function 2000+c,
light and cameras 3000+c, path-tracer key 4000+c.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

U8, U16, F32 = 0, 1, 2
DIRECTIONAL, AREA = 0, 1

Vec3 = Tuple[float, float, float]


@dataclass
class Volume:
    data: np.ndarray          # 1-D, storage order (x-fastest, or 8^3 brick-major)
    vtype: int                # U8 / U16 / F32
    dims: Tuple[int, int, int]
    brick: int                # 0 linear, 8 bricked
    vmin: float
    vmax: float
    box_min: Vec3 = (-1.0, -1.0, -1.0)
    box_max: Vec3 = (1.0, 1.0, 1.0)


@dataclass
class Medium:
    lut: np.ndarray           # float32 [lut_size, 4] RGBA
    scale: float              # density scale (sigma_t = scale * alpha), per world unit


@dataclass
class Light:
    kind: int                 # DIRECTIONAL / AREA
    dir: Vec3 = (0.0, 0.0, 1.0)
    corner: Vec3 = (0.0, 0.0, 0.0)
    e1: Vec3 = (0.0, 0.0, 0.0)
    e2: Vec3 = (0.0, 0.0, 0.0)
    radiance: Vec3 = (1.0, 1.0, 1.0)
    env: Vec3 = (0.0, 0.0, 0.0)


@dataclass
class Params:
    M: int
    N: int
    center: Vec3 = (0.0, 0.0, 0.0)
    radius: float = math.sqrt(3.0)
    spp: int = 16
    max_bounces: int = 4
    g: float = 0.0
    majorant: float = 0.0     # <= 0: 1.25 * scale * max alpha
    grid: int = 0             # majorant grid cells per axis (0: one global majorant)
    surface: int = 0          # 1: isosurface variant at raw value iso
    iso: float = 0.0
    seed: int = 0
    jitter: int = 1
    origin_rows: int = 0      # 0: all M origins; M // 2: upper hemisphere only


@dataclass
class Camera:
    eye: Vec3
    target: Vec3
    up: Vec3
    vfov: float


@dataclass
class Scene:
    name: str
    volume: Volume
    medium: Medium
    light: Light
    params: Params
    cams: List[Camera] = field(default_factory=list)
    width: int = 0
    height: int = 0
    K: int = 5

    def replace(self, **kw) -> "Scene":
        return dataclasses.replace(self, **kw)

    def with_params(self, **kw) -> "Scene":
        return dataclasses.replace(self, params=dataclasses.replace(self.params, **kw))


# --------------------------------------------------------------------------
# random helpers
# --------------------------------------------------------------------------
def _rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly random rotation matrix (QR of a Gaussian matrix, sign-fixed)."""
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def brick_layout(vol_zyx: np.ndarray, b: int = 8) -> np.ndarray:
    """Reorder a (nz, ny, nx) array into b^3 bricks, brick-major with bricks
    ordered x-fastest and voxels x-fastest inside each brick."""
    nz, ny, nx = vol_zyx.shape
    assert nx % b == 0 and ny % b == 0 and nz % b == 0
    v = vol_zyx.reshape(nz // b, b, ny // b, b, nx // b, b)
    # axes: (bz, z, by, y, bx, x) -> (bz, by, bx, z, y, x)
    return np.ascontiguousarray(v.transpose(0, 2, 4, 1, 3, 5)).reshape(-1)


# --------------------------------------------------------------------------
# volumes
# --------------------------------------------------------------------------
def blob_volume(n: int, seed: int, nblobs: int = 8) -> np.ndarray:
    """Sum of anisotropic Gaussian blobs on an n^3 grid, normalised to max 1.

    Centres uniform in the central 60 % of the grid, per-axis sigma uniform in
    [3, 12] voxels at n = 64 (scaled by n / 64), random rotation, amplitude
    uniform in [0.5, 1].  Returned as float64 (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    s = n / 64.0
    idx = np.arange(n, dtype=np.float64) + 0.5
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    pts = np.stack([x, y, z], -1)
    vol = np.zeros((n, n, n))
    for _ in range(nblobs):
        c = rng.uniform(0.2 * n, 0.8 * n, 3)
        sig = rng.uniform(3.0, 12.0, 3) * s
        rot = _rotation(rng)
        amp = rng.uniform(0.5, 1.0)
        d = (pts - c) @ rot
        vol += amp * np.exp(-0.5 * np.sum((d / sig) ** 2, -1))
    return vol / vol.max()


def phantom_volume(n: int, seed: int, n_ellipsoids: int, noise: float = 20.0,
                   chunk: int = 64) -> np.ndarray:
    """CT-like phantom: nested random ellipsoids with HU values, as uint16.

    Ellipsoid 0 is centred near the grid centre with semi-axes 0.6-0.95 of
    the half extent.  Every later ellipsoid picks a random existing parent and
    lies inside it: semi-axes 0.5-0.9 x the parent's smallest semi-axis,
    centre offset within the remaining margin, random rotation.  HU of the
    outer shell (the body) uniform in [-100, 300], of every inner shell
    uniform in [-1000, 2000]; background -1000, Gaussian noise sigma = 20 HU;
    stored as clamp(round(HU + 1024), 0, 65535).  Returned (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    half = n / 2.0
    ells = []  # (centre, rotation, semi-axes, HU)
    c0 = np.full(3, half) + rng.uniform(-0.05, 0.05, 3) * n
    a0 = rng.uniform(0.6, 0.95, 3) * (half - np.abs(c0 - half).max())
    ells.append((c0, _rotation(rng), a0, rng.uniform(-100.0, 300.0)))  # body: soft tissue
    for _ in range(1, n_ellipsoids):
        pc, prot, pa, _ = ells[rng.integers(len(ells))]
        a = rng.uniform(0.5, 0.9, 3) * pa.min()
        margin = pa.min() - a.max()
        off = _unit(rng) * margin * rng.uniform(0.0, 1.0) ** (1.0 / 3.0)
        ells.append((pc + off, _rotation(rng), a, rng.uniform(-1000.0, 2000.0)))
    out = np.empty((n, n, n), dtype=np.uint16)
    idx = np.arange(n, dtype=np.float32) + 0.5
    for z0 in range(0, n, chunk):
        z1 = min(n, z0 + chunk)
        hu = np.full((z1 - z0, n, n), -1000.0, dtype=np.float32)
        for c, rot, a, h in ells:
            r = a.max()
            if c[2] + r < z0 or c[2] - r > z1:
                continue
            zlo, zhi = max(z0, int(c[2] - r) - 1), min(z1, int(c[2] + r) + 2)
            ylo, yhi = max(0, int(c[1] - r) - 1), min(n, int(c[1] + r) + 2)
            xlo, xhi = max(0, int(c[0] - r) - 1), min(n, int(c[0] + r) + 2)
            if zlo >= zhi:
                continue
            dz = (idx[zlo:zhi] - c[2])[:, None, None]
            dy = (idx[ylo:yhi] - c[1])[None, :, None]
            dx = (idx[xlo:xhi] - c[0])[None, None, :]
            q = np.zeros((zhi - zlo, yhi - ylo, xhi - xlo), dtype=np.float32)
            for k in range(3):  # rotated coordinate k over its semi-axis
                q += ((rot[0, k] * dx + rot[1, k] * dy + rot[2, k] * dz) / a[k]).astype(np.float32) ** 2
            hu[zlo - z0:zhi - z0, ylo:yhi, xlo:xhi][q <= 1.0] = h
        hu += rng.standard_normal(hu.shape, dtype=np.float32) * noise
        out[z0:z1] = np.clip(np.rint(hu + 1024.0), 0, 65535).astype(np.uint16)
    return out


# --------------------------------------------------------------------------
# transfer function, lights, cameras
# --------------------------------------------------------------------------
def transfer_lut(seed: int, size: int = 256, knots: int = 6) -> np.ndarray:
    """Piecewise-linear RGBA table through `knots` random knots at normalised
    positions 0, sorted interior positions and 1; RGBA uniform in [0, 1] with
    alpha = 0 at the first knot (transparent background)."""
    rng = np.random.default_rng(seed)
    pos = np.concatenate([[0.0], np.sort(rng.uniform(0.0, 1.0, knots - 2)), [1.0]])
    val = rng.uniform(0.0, 1.0, (knots, 4))
    val[0, 3] = 0.0
    s = np.arange(size) / (size - 1)
    lut = np.stack([np.interp(s, pos, val[:, c]) for c in range(4)], -1)
    return lut.astype(np.float32)


def directional_light(seed: int) -> Light:
    rng = np.random.default_rng(seed)
    d = _unit(rng)
    return Light(kind=DIRECTIONAL, dir=tuple(d), radiance=(1.0, 1.0, 1.0))


def area_light(seed: int, radius: float, center: Vec3 = (0.0, 0.0, 0.0)) -> Light:
    """Square of side R at distance 2R from O along a random direction,
    facing O, radiance 4 (irradiance at O close to 1)."""
    rng = np.random.default_rng(seed)
    u = _unit(rng)
    t1 = np.cross(u, [0.0, 0.0, 1.0] if abs(u[2]) < 0.9 else [1.0, 0.0, 0.0])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(t1, u)  # cross(t1, t2) = -u: emitting side faces O
    c = np.asarray(center) + 2.0 * radius * u
    corner = c - 0.5 * radius * (t1 + t2)
    return Light(kind=AREA, corner=tuple(corner), e1=tuple(radius * t1), e2=tuple(radius * t2),
                 radiance=(4.0, 4.0, 4.0))


def cameras(seed: int, count: int, radius: float, center: Vec3 = (0.0, 0.0, 0.0)) -> List[Camera]:
    """Eyes at distance uniform in [2.5R, 4R], direction uniform on the
    sphere, looking at O, vertical FOV 2 asin(R / dist) * 1.05."""
    rng = np.random.default_rng(seed + 7919)
    out = []
    for _ in range(count):
        d = _unit(rng)
        dist = rng.uniform(2.5, 4.0) * radius
        eye = np.asarray(center) + dist * d
        up = (0.0, 0.0, 1.0) if abs(d[2]) < 0.99 else (1.0, 0.0, 0.0)
        out.append(Camera(eye=tuple(eye), target=tuple(center), up=up,
                          vfov=2.0 * math.asin(radius / dist) * 1.05))
    return out


def seam_cameras(radius: float, center: Vec3 = (0.0, 0.0, 0.0)) -> List[Camera]:
    """Three views from near the equator plane (elevations 0.15, -0.2, 0 rad)
    at distance 3R: their front hits cover both hemispheres of S and the seam
    between them (cases for a light field that stores only the upper half of
    the origins)."""
    out = []
    for az, el in ((0.3, 0.15), (2.1, -0.2), (4.0, 0.0)):
        d = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
        out.append(Camera(eye=tuple(np.asarray(center) + 3.0 * radius * d), target=tuple(center),
                          up=(0.0, 0.0, 1.0), vfov=2.0 * math.asin(1.0 / 3.0) * 1.05))
    return out


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
_VOL_CACHE: dict = {}


def _blob(n: int, seed: int, vtype: int) -> Volume:
    key = ("blob", n, seed, vtype)
    if key not in _VOL_CACHE:
        v = blob_volume(n, seed)
        if vtype == U8:
            data = np.rint(v * 255.0).astype(np.uint8).reshape(-1)
            _VOL_CACHE[key] = Volume(data, U8, (n, n, n), 0, 0.0, 255.0)
        else:
            data = v.astype(np.float32).reshape(-1)
            _VOL_CACHE[key] = Volume(data, F32, (n, n, n), 0, 0.0, 1.0)
    return _VOL_CACHE[key]


def _phantom(n: int, seed: int, nell: int, brick: int) -> Volume:
    key = ("phantom", n, seed, nell, brick)
    if key not in _VOL_CACHE:
        v = phantom_volume(n, seed, nell)
        data = brick_layout(v, 8) if brick == 8 else v.reshape(-1)
        # LUT window HU [-1000, 2000] in stored units (HU + 1024)
        _VOL_CACHE[key] = Volume(data, U16, (n, n, n), brick, 24.0, 3024.0)
    return _VOL_CACHE[key]


def config(c: int, **over) -> Scene:
    """Workload c (1..5) at its full size.  Keyword overrides replace run
    parameters (M, N, spp, max_bounces, ...) or view settings (views, width,
    height, K) so tests can run the same scene at smaller sizes.  Every
    workload tracks against a majorant grid, G^3 cells with G measured
    fastest on MI355X for that workload (grid=0 selects the global
    majorant)."""
    R = math.sqrt(3.0)
    views = over.pop("views", None)
    width = over.pop("width", None)
    height = over.pop("height", None)
    K = over.pop("K", 5)
    vol_n = over.pop("vol_n", None)
    if c == 1:
        vol = _blob(vol_n or 64, 1001, U8)
        lt = directional_light(3001)
        prm = Params(M=256, N=256, radius=R, spp=16, max_bounces=4, g=0.0, seed=4001, grid=4)
        nv, w, h = 4, 64, 48
    elif c == 2:
        vol = _phantom(vol_n or 256, 1002, 12, 0)
        lt = area_light(3002, R)
        prm = Params(M=2048, N=2048, radius=R, spp=64, max_bounces=8, g=0.3, seed=4002, grid=5)
        nv, w, h = 32, 1920, 1080
    elif c in (3, 4):
        vol = _phantom(vol_n or 512, 1003, 40, 8)
        lt = area_light(3003 if c == 3 else 3004, R)
        if c == 3:
            prm = Params(M=8192, N=8192, radius=R, spp=128, max_bounces=8, g=0.3, seed=4003, grid=8)
        else:
            prm = Params(M=32768, N=32768, radius=R, spp=16, max_bounces=8, g=0.3, seed=4004, grid=8)
        nv, w, h = 4, 512, 512
    elif c == 5:
        vol = _blob(vol_n or 128, 1005, F32)
        lt = directional_light(3005)
        prm = Params(M=1024, N=1024, radius=R, spp=32, max_bounces=4, g=0.0, seed=4005, grid=8)
        nv, w, h = 16, 512, 512
    else:
        raise ValueError(f"unknown workload {c}")
    med = Medium(lut=transfer_lut(2000 + c), scale=10.0)
    prm = dataclasses.replace(prm, **over)
    nv = views if views is not None else nv
    cams = cameras(3000 + c, nv, R)
    return Scene(name=f"c{c}", volume=vol, medium=med, light=lt, params=prm, cams=cams,
                 width=width or w, height=height or h, K=K)


def target_medium(scene: Scene, seed: int = 6005) -> Medium:
    """Perturbed medium used to render seeded target views for the
    differentiation workload: LUT entries +- 0.1 (clamped to [0, 1], alpha of
    entry 0 kept at 0) and density scale x 1.2."""
    rng = np.random.default_rng(seed)
    lut = scene.medium.lut + rng.uniform(-0.1, 0.1, scene.medium.lut.shape).astype(np.float32)
    lut = np.clip(lut, 0.0, 1.0).astype(np.float32)
    lut[0, 3] = 0.0
    return Medium(lut=lut, scale=scene.medium.scale * 1.2)


def constant_volume(n: int = 8, value: float = 1.0) -> Volume:
    """Homogeneous f32 volume (for closed-form checks)."""
    return Volume(np.full(n * n * n, value, dtype=np.float32), F32, (n, n, n), 0, 0.0, 1.0)


def constant_lut(rgb: Vec3, alpha: float, size: int = 2) -> np.ndarray:
    lut = np.zeros((size, 4), dtype=np.float32)
    lut[:, :3] = rgb
    lut[:, 3] = alpha
    return lut


def random_rays(M: int, N: int, count: int, seed: int, exclude_degenerate: bool = True) -> np.ndarray:
    """Seeded sample of distinct ray indices k = i*N + j (sorted)."""
    rng = np.random.default_rng(seed)
    total = M * N
    count = min(count, total)
    if count * 4 > total:
        ks = rng.permutation(total)[:count]
    else:
        ks = np.unique(rng.integers(0, total, int(count * 1.2) + 16))
        rng.shuffle(ks)
        ks = ks[:count]
    ks = np.sort(ks).astype(np.int64)
    if exclude_degenerate and M == N:
        ks = ks[(ks // N) != (ks % N)]
    return ks
