"""Seeded synthetic range images standing in for the paper's datasets.

The paper evaluates on 480x640 depth images rendered from meshes, on real
depth (DIODE, ScanNet) and on stereo disparity (Sec. IV-A); none of that data
is available here.  This module ray-casts analytic primitives (planes, spheres,
oriented boxes) through a pinhole camera (the projection of Sec. III,
eq. intrinisc_matrix) and returns the raw range image, the analytic surface
normal at every hit and a region id.  It holds no part of the estimator: both
the HIP path and the FP64 oracle consume what it produces.

Rendering runs on whatever torch device is asked for (CPU for tests, the GPU
for large benchmark batches); every random draw comes from a seeded numpy
generator (scene layout) or a seeded torch generator on that device (noise,
holes), so a (recipe, seed, device) triple always yields the same image.

Recipes (sizes, intrinsics and value ranges of the workloads):
  * ``indoor``   - 480x640 FP32 depth, fx=fy=481.2, principal point at the
    image centre, back wall + 2 planes + 2 spheres, depth 0.5-5 m, no noise.
  * ``cluttered`` - planes, spheres and oriented boxes; optional multiplicative
    Gaussian depth noise and Bernoulli zero-depth holes.
  * ``road``     - 375x1242 stereo disparity, f=721.5, baseline 0.54 m, road
    plane plus box obstacles and side walls; disparity 1-128 px, sky and
    out-of-range pixels are 0, +-0.25 px uniform noise.
  * ``depth_mm_u16`` - the cluttered recipe at any size, stored as uint16
    millimetres (0 = invalid).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

__all__ = [
    "Camera", "camera_for", "render", "indoor_scene", "cluttered_scene",
    "road_scene", "Frame", "make_indoor", "make_cluttered", "make_road",
    "make_u16", "uneven_sizes", "INDOOR_K",
]

INDOOR_K = (481.2, 481.2, 319.5, 239.5)


@dataclass(frozen=True)
class Camera:
    H: int
    W: int
    fx: float
    fy: float
    u0: float
    v0: float

    def as_tuple(self) -> Tuple[float, float, float, float]:
        return (self.fx, self.fy, self.u0, self.v0)


def camera_for(H: int, W: int, f640: float = 481.2) -> Camera:
    """Pinhole camera with the indoor focal length scaled to the image width
    and the principal point at the image centre."""
    f = f640 * W / 640.0
    return Camera(H, W, f, f, (W - 1) / 2.0, (H - 1) / 2.0)


# --------------------------------------------------------------------------
# primitives
# --------------------------------------------------------------------------

def _unit(x):
    x = np.asarray(x, dtype=np.float64)
    return x / np.linalg.norm(x)


def _dir_in_cone(rng: np.random.Generator, cone_deg: float) -> np.ndarray:
    """Unit vector drawn uniformly from the spherical cap of half-angle
    ``cone_deg`` around -z (towards the camera)."""
    c = rng.uniform(math.cos(math.radians(cone_deg)), 1.0)
    s = math.sqrt(max(0.0, 1.0 - c * c))
    a = rng.uniform(0.0, 2.0 * math.pi)
    return np.array([s * math.cos(a), s * math.sin(a), -c])


def _rot(axis, ang):
    axis = _unit(axis)
    x, y, z = axis
    c, s = math.cos(ang), math.sin(ang)
    C = 1 - c
    return np.array([[c + x * x * C, x * y * C - z * s, x * z * C + y * s],
                     [y * x * C + z * s, c + y * y * C, y * z * C - x * s],
                     [z * x * C - y * s, z * y * C + x * s, c + z * z * C]])


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _ray_at(cam: Camera, u: float, v: float) -> np.ndarray:
    return np.array([(u - cam.u0) / cam.fx, (v - cam.v0) / cam.fy, 1.0])


def _plane(n, b):
    return {"type": "plane", "n": np.asarray(n, dtype=np.float64), "b": float(b)}


def _sphere(c, R):
    return {"type": "sphere", "c": np.asarray(c, dtype=np.float64), "R": float(R)}


def _box(c, Rm, h):
    return {"type": "box", "c": np.asarray(c, dtype=np.float64),
            "Rm": np.asarray(Rm, dtype=np.float64), "h": np.asarray(h, dtype=np.float64)}


# --------------------------------------------------------------------------
# ray casting
# --------------------------------------------------------------------------

def _intersect(p, dx, dy, need_normal):
    """Return (t, normal or None) for rays d = (dx, dy, 1); t = inf on miss.
    Because d_z = 1 the ray parameter t is the depth z of the hit."""
    inf = torch.tensor(float("inf"), dtype=dx.dtype, device=dx.device)
    if p["type"] == "plane":
        n = p["n"]
        nd = n[0] * dx + n[1] * dy + n[2]
        t = -p["b"] / nd
        t = torch.where(nd != 0, t, inf)
        nrm = None
        if need_normal:
            sgn = torch.where(nd < 0, 1.0, -1.0).to(dx.dtype)  # camera-facing
            nrm = torch.stack([sgn * n[0], sgn * n[1], sgn * n[2]])
        return t, nrm
    if p["type"] == "sphere":
        c, R = p["c"], p["R"]
        a = dx * dx + dy * dy + 1.0
        bq = c[0] * dx + c[1] * dy + c[2]
        cq = float(c @ c) - R * R
        disc = bq * bq - a * cq
        ok = disc >= 0
        t = (bq - torch.sqrt(torch.clamp(disc, min=0.0))) / a
        t = torch.where(ok, t, inf)
        nrm = None
        if need_normal:
            nrm = torch.stack([(t * dx - c[0]) / R, (t * dy - c[1]) / R, (t - c[2]) / R])
        return t, nrm
    if p["type"] == "box":
        c, Rm, h = p["c"], p["Rm"], p["h"]
        # ray origin and direction in the box frame (columns of Rm = box axes)
        o = -(Rm.T @ c)
        d = [Rm[0, k] * dx + Rm[1, k] * dy + Rm[2, k] for k in range(3)]
        tnear = torch.full_like(dx, -float("inf"))
        tfar = torch.full_like(dx, float("inf"))
        axis = torch.zeros_like(dx, dtype=torch.int64)
        for k in range(3):
            dk = d[k]
            safe = torch.where(dk != 0, dk, torch.ones_like(dk))
            t1 = (-h[k] - o[k]) / safe
            t2 = (h[k] - o[k]) / safe
            lo = torch.minimum(t1, t2)
            hi = torch.maximum(t1, t2)
            # a ray parallel to the slab is either always inside it or never
            if -h[k] <= o[k] <= h[k]:
                lo_par, hi_par = -float("inf"), float("inf")
            else:
                lo_par, hi_par = float("inf"), -float("inf")
            lo = torch.where(dk != 0, lo, torch.full_like(lo, lo_par))
            hi = torch.where(dk != 0, hi, torch.full_like(hi, hi_par))
            upd = lo > tnear
            axis = torch.where(upd, k, axis)
            tnear = torch.maximum(tnear, lo)
            tfar = torch.minimum(tfar, hi)
        hit = (tnear <= tfar) & (tnear > 0)
        t = torch.where(hit, tnear, inf)
        nrm = None
        if need_normal:
            comps = []
            dsel = torch.where(axis == 0, d[0], torch.where(axis == 1, d[1], d[2]))
            sgn = torch.where(dsel > 0, -1.0, 1.0).to(dx.dtype)
            for r in range(3):
                col = torch.where(axis == 0, Rm[r, 0], torch.where(axis == 1, Rm[r, 1], Rm[r, 2]))
                comps.append(sgn * col)
            nrm = torch.stack(comps)
        return t, nrm
    raise ValueError(p["type"])


def render(prims, cam: Camera, znear: float, zfar: float, device="cpu",
           need_gt: bool = True):
    """Nearest hit with znear <= z <= zfar for every pixel.

    Returns (depth float64 [H,W] with 0 where nothing is hit,
             normals float64 [3,H,W] or None, region int16 [H,W] (-1 = none)).
    Pixel centres sit at integer (u, v), u along columns and v along rows."""
    dev = torch.device(device)
    v = torch.arange(cam.H, dtype=torch.float64, device=dev).view(-1, 1)
    u = torch.arange(cam.W, dtype=torch.float64, device=dev).view(1, -1)
    dx = ((u - cam.u0) / cam.fx).expand(cam.H, cam.W)
    dy = ((v - cam.v0) / cam.fy).expand(cam.H, cam.W)
    best = torch.full((cam.H, cam.W), float("inf"), dtype=torch.float64, device=dev)
    region = torch.full((cam.H, cam.W), -1, dtype=torch.int16, device=dev)
    nrm = torch.zeros((3, cam.H, cam.W), dtype=torch.float64, device=dev) if need_gt else None
    for i, p in enumerate(prims):
        t, n = _intersect(p, dx, dy, need_gt)
        take = (t >= znear) & (t <= zfar) & (t < best)
        best = torch.where(take, t, best)
        region = torch.where(take, torch.tensor(i, dtype=torch.int16, device=dev), region)
        if need_gt:
            nrm = torch.where(take.unsqueeze(0), n, nrm)
    depth = torch.where(torch.isinf(best), torch.zeros_like(best), best)
    return depth, nrm, region


# --------------------------------------------------------------------------
# scene recipes (layout only; numpy RNG)
# --------------------------------------------------------------------------

def _back_wall(rng, cam: Camera, znear, zfar, z_lo=3.0, z_hi=4.5, cone=30.0):
    """A plane that covers the whole view with depth inside [znear, zfar]."""
    corners = [(0, 0), (cam.W - 1, 0), (0, cam.H - 1), (cam.W - 1, cam.H - 1)]
    for _ in range(1000):
        n = _dir_in_cone(rng, cone)
        z0 = rng.uniform(z_lo, z_hi)
        b = -n[2] * z0                      # passes through (0, 0, z0)
        ok = True
        for (u, v) in corners:
            d = _ray_at(cam, u, v)
            nd = float(n @ d)
            if nd >= 0:
                ok = False
                break
            z = -b / nd
            if not (znear + 0.05 <= z <= zfar - 0.05):
                ok = False
                break
        if ok:
            return _plane(n, b)
    raise RuntimeError("could not place a back wall")


def _plane_through_pixel(rng, cam, cone, z_lo, z_hi):
    n = _dir_in_cone(rng, cone)
    u = rng.uniform(0, cam.W - 1)
    v = rng.uniform(0, cam.H - 1)
    p0 = rng.uniform(z_lo, z_hi) * _ray_at(cam, u, v)
    return _plane(n, -float(n @ p0))


def _sphere_at_pixel(rng, cam, z_lo, z_hi, r_lo, r_hi):
    u = rng.uniform(0.1 * cam.W, 0.9 * cam.W)
    v = rng.uniform(0.1 * cam.H, 0.9 * cam.H)
    c = rng.uniform(z_lo, z_hi) * _ray_at(cam, u, v)
    return _sphere(c, rng.uniform(r_lo, r_hi))


def _box_at_pixel(rng, cam, z_lo, z_hi, h_lo, h_hi):
    u = rng.uniform(0.1 * cam.W, 0.9 * cam.W)
    v = rng.uniform(0.1 * cam.H, 0.9 * cam.H)
    c = rng.uniform(z_lo, z_hi) * _ray_at(cam, u, v)
    return _box(c, _random_rotation(rng), rng.uniform(h_lo, h_hi, size=3))


def indoor_scene(seed: int, cam: Camera):
    """Back wall + 2 random planes (normals within 60 deg of -z, through a
    point 2-4.5 m deep) + 2 spheres (centre depth 1.2-2.5 m, radius
    0.2-0.6 m); visible depth 0.5-5 m."""
    rng = np.random.default_rng(seed)
    prims = [_back_wall(rng, cam, 0.5, 5.0)]
    for _ in range(2):
        prims.append(_plane_through_pixel(rng, cam, 60.0, 2.0, 4.5))
    for _ in range(2):
        prims.append(_sphere_at_pixel(rng, cam, 1.2, 2.5, 0.2, 0.6))
    return prims, 0.5, 5.0


def cluttered_scene(seed: int, cam: Camera):
    """Back wall + 1-2 planes + 1-3 spheres + 1-3 oriented boxes."""
    rng = np.random.default_rng(seed)
    prims = [_back_wall(rng, cam, 0.5, 5.0)]
    for _ in range(int(rng.integers(1, 3))):
        prims.append(_plane_through_pixel(rng, cam, 60.0, 2.0, 4.5))
    for _ in range(int(rng.integers(1, 4))):
        prims.append(_sphere_at_pixel(rng, cam, 1.0, 2.8, 0.15, 0.6))
    for _ in range(int(rng.integers(1, 4))):
        prims.append(_box_at_pixel(rng, cam, 1.0, 2.8, 0.1, 0.5))
    return prims, 0.5, 5.0


def road_scene(seed: int, cam: Camera):
    """Road plane (camera 1.5-1.8 m above it, +-2 deg pitch/roll), 3-8 box
    obstacles standing on it and 0-2 side walls.  y points down."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(1.5, 1.8)
    R_road = _rot([1, 0, 0], math.radians(rng.uniform(-2, 2))) @ \
        _rot([0, 0, 1], math.radians(rng.uniform(-2, 2)))
    up = R_road @ np.array([0.0, -1.0, 0.0])          # road normal, towards camera
    prims = [_plane(up, h)]                            # up . p + h = 0
    for _ in range(int(rng.integers(0, 3))):
        side = -1.0 if rng.uniform() < 0.5 else 1.0
        wn = _rot([0, 1, 0], math.radians(rng.uniform(-20, 20))) @ np.array([-side, 0.0, 0.0])
        x0 = side * rng.uniform(6.0, 15.0)
        prims.append(_plane(wn, -float(wn @ np.array([x0, 0.0, 20.0]))))
    for _ in range(int(rng.integers(3, 9))):
        hx, hy, hz = rng.uniform(0.3, 1.5), rng.uniform(0.5, 1.5), rng.uniform(0.3, 2.0)
        q = np.array([rng.uniform(-8, 8), h, rng.uniform(6, 60)])
        q = q - (float(up @ q) + h) * up                    # foot point on the road
        c = q + hy * up
        Rm = R_road @ _rot([0, 1, 0], rng.uniform(0, 2 * math.pi))
        prims.append(_box(c, Rm, [hx, hy, hz]))
    return prims, 0.05, 1e4


# --------------------------------------------------------------------------
# image makers
# --------------------------------------------------------------------------

@dataclass
class Frame:
    raw: torch.Tensor                 # [H,W] float32 / uint16 / float16
    cam: Camera
    kind: str                         # "depth" or "disparity"
    gt: Optional[torch.Tensor] = None  # [3,H,W] float64 analytic normals
    region: Optional[torch.Tensor] = None
    depth64: Optional[torch.Tensor] = None  # noiseless float64 depth


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    return g


def make_indoor(seed: int = 0, cam: Optional[Camera] = None, device="cpu",
                need_gt=True) -> Frame:
    cam = cam or Camera(480, 640, *INDOOR_K)
    prims, zn, zf = indoor_scene(seed, cam)
    d64, gt, reg = render(prims, cam, zn, zf, device, need_gt)
    return Frame(d64.to(torch.float32), cam, "depth", gt, reg, d64)


def make_cluttered(seed: int, cam: Optional[Camera] = None, device="cpu",
                   noise: float = 0.005, holes: float = 0.03, need_gt=False) -> Frame:
    """FP32 depth: z * (1 + noise * N(0,1)), then Bernoulli(holes) -> 0."""
    cam = cam or Camera(480, 640, *INDOOR_K)
    prims, zn, zf = cluttered_scene(seed, cam)
    d64, gt, reg = render(prims, cam, zn, zf, device, need_gt)
    g = _gen(seed * 7919 + 1, device)
    z = d64
    if noise > 0:
        z = z * (1.0 + noise * torch.randn(z.shape, generator=g, dtype=torch.float64, device=z.device))
    if holes > 0:
        z = torch.where(torch.rand(z.shape, generator=g, dtype=torch.float64, device=z.device) < holes,
                        torch.zeros_like(z), z)
    return Frame(z.to(torch.float32), cam, "depth", gt, reg, d64)


ROAD_CAM = Camera(375, 1242, 721.5, 721.5, 620.5, 187.0)
ROAD_BASELINE = 0.54


def make_road(seed: int, cam: Optional[Camera] = None, device="cpu",
              noise: float = 0.25, need_gt=False) -> Frame:
    """FP32 disparity d = f * baseline / z kept where 1 <= d <= 128 (else 0),
    plus U(-noise, noise) px on the kept pixels."""
    cam = cam or ROAD_CAM
    prims, zn, zf = road_scene(seed, cam)
    d64, gt, reg = render(prims, cam, zn, zf, device, need_gt)
    disp = torch.where(d64 > 0, cam.fx * ROAD_BASELINE / torch.where(d64 > 0, d64, torch.ones_like(d64)),
                       torch.zeros_like(d64))
    ok = (disp >= 1.0) & (disp <= 128.0)
    disp = torch.where(ok, disp, torch.zeros_like(disp))
    if noise > 0:
        g = _gen(seed * 7919 + 2, device)
        jitter = (torch.rand(disp.shape, generator=g, dtype=torch.float64, device=disp.device) * 2 - 1) * noise
        disp = torch.where(ok, disp + jitter, disp)
    return Frame(disp.to(torch.float32), cam, "disparity", gt, reg, d64)


def make_u16(seed: int, cam: Camera, device="cpu", noise: float = 0.005,
             holes: float = 0.03, need_gt=False) -> Frame:
    """uint16 millimetre depth of the cluttered recipe: round(1000 z), with the
    same multiplicative noise and holes; 0 = invalid."""
    fr = make_cluttered(seed, cam, device, noise=0.0, holes=0.0, need_gt=need_gt)
    g = _gen(seed * 7919 + 3, device)
    z = fr.depth64
    if noise > 0:
        z = z * (1.0 + noise * torch.randn(z.shape, generator=g, dtype=torch.float64, device=z.device))
    mm = torch.clamp(torch.round(z * 1000.0), 0, 65535)
    if holes > 0:
        mm = torch.where(torch.rand(z.shape, generator=g, dtype=torch.float64, device=z.device) < holes,
                         torch.zeros_like(mm), mm)
    # int32 -> int16 keeps the low 16 bits; viewing them as uint16 is the
    # value (a path every torch device supports)
    u16 = mm.to(torch.int32).to(torch.int16).view(torch.uint16)
    return Frame(u16, cam, "depth", fr.gt, fr.region, fr.depth64)


UNEVEN_SHAPES = ((240, 320), (480, 640), (720, 1280), (1080, 1920))


def uneven_sizes(n: int, seed: int = 3999,
                 shapes: Sequence[Tuple[int, int]] = UNEVEN_SHAPES) -> List[Tuple[int, int]]:
    """n frame shapes drawn uniformly from ``shapes``."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(shapes), size=n)
    return [tuple(shapes[i]) for i in idx]


def uneven_batch(n: int, seed: int = 3999, scenes_per_shape: int = 16, device="cpu"):
    """The uneven-batch workload: n uint16 millimetre depth frames with shapes
    from ``uneven_sizes(n, seed)``, ``scenes_per_shape`` distinct scenes per
    shape reused across the batch.  Returns (shapes, Ks, k_index, frames):
    Ks holds one intrinsics tuple per distinct shape (sorted), k_index the
    row of Ks of each frame."""
    shapes = uneven_sizes(n, seed=seed)
    uniq = sorted(set(shapes))
    cams = {sh: camera_for(*sh) for sh in uniq}
    pool = {sh: [make_u16(seed + 1 + 97 * j + i, cams[sh], device=device).raw
                 for j in range(scenes_per_shape)] for i, sh in enumerate(uniq)}
    kidx = {sh: i for i, sh in enumerate(uniq)}
    frames = [pool[sh][k % scenes_per_shape] for k, sh in enumerate(shapes)]
    return shapes, [cams[sh].as_tuple() for sh in uniq], [kidx[sh] for sh in shapes], frames
