"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module only *builds inputs*: analytic scenes (a box room with spheres and
boxes, optional emitters), pinhole cameras, probe-grid layouts and the fixed
parameters of each workload.  It contains none of the method's arithmetic
(no ray tracing, probe queries, sampling or resampling).  Every array it
returns is float32/uint32, so both implementations start from bit-identical
values: the GPU reads them directly, the oracle reads their exact float64
conversions.

The paper evaluates on its own six indoor scenes at 1920x1080 and one sample
per pixel (Sec. 4); those assets are not available, so seeded box rooms with
the same character (indoor, multi-bounce diffuse, a few small bright emitters)
stand in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

PRIM_SPHERE = 0
PRIM_BOX = 1
PRIM_RECORD = 16          # floats per primitive record (64 bytes)
MISS = 0xFFFFFFFF


# --------------------------------------------------------------------------
# primitive records
# --------------------------------------------------------------------------
def prim_records(types, centers, sizes, albedo, emit, spec=None, rough=None) -> np.ndarray:
    """Pack primitives into the 64-byte record layout used by the C ABI:
    [cx cy cz type | sx sy sz 0 | ar ag ab ks | er eg eb alpha] (type as uint32
    bits; spheres keep their radius in sx; ks the grey weight of a GGX
    specular layer of roughness alpha, 0 for a Lambertian surface)."""
    n = len(types)
    rec = np.zeros((n, PRIM_RECORD), dtype=np.float32)
    rec[:, 0:3] = np.asarray(centers, dtype=np.float32).reshape(n, 3)
    rec.view(np.uint32)[:, 3] = np.asarray(types, dtype=np.uint32)
    rec[:, 4:7] = np.asarray(sizes, dtype=np.float32).reshape(n, 3)
    rec[:, 8:11] = np.asarray(albedo, dtype=np.float32).reshape(n, 3)
    rec[:, 12:15] = np.asarray(emit, dtype=np.float32).reshape(n, 3)
    if spec is not None:
        rec[:, 11] = np.asarray(spec, dtype=np.float32).reshape(n)
        rec[:, 15] = np.asarray(rough, dtype=np.float32).reshape(n)
    return rec


@dataclasses.dataclass
class Scene:
    prims: np.ndarray                 # (n, 16) float32 records
    has_room: bool
    room_lo: np.ndarray               # (3,) float32
    room_hi: np.ndarray
    wall_albedo: np.ndarray
    sky: np.ndarray                   # radiance of rays that leave the scene
    eps: float                        # ray-origin offset along the surface normal
    wall_emit: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros(3, np.float32))   # radiance emitted by the walls

    @property
    def n_prims(self) -> int:
        return int(self.prims.shape[0])

    def bounds(self):
        if self.has_room:
            return self.room_lo.copy(), self.room_hi.copy()
        c = self.prims[:, 0:3]
        s = self.prims[:, 4:7].copy()
        t = self.prims.view(np.uint32)[:, 3]
        s[t == PRIM_SPHERE, 1] = s[t == PRIM_SPHERE, 0]
        s[t == PRIM_SPHERE, 2] = s[t == PRIM_SPHERE, 0]
        return (c - s).min(0).astype(np.float32), (c + s).max(0).astype(np.float32)


@dataclasses.dataclass
class Camera:
    eye: np.ndarray
    fwd: np.ndarray
    right: np.ndarray
    up: np.ndarray
    tan_half_fovy: float
    width: int
    height: int


@dataclasses.dataclass
class ProbeGrid:
    dims: tuple                       # (nx, ny, nz)
    lo: np.ndarray                    # grid origin; probe (i,j,k) sits at lo + (idx+0.5)*spacing
    spacing: np.ndarray
    irr_res: int = 8                  # interior octahedral texels per side (irradiance)
    dep_res: int = 16                 # interior octahedral texels per side (depth moments)
    bias_dist: float = 0.0            # view-path bias distance d (0.3 x min spacing)
    var_floor: float = 0.0            # Chebyshev variance floor (1e-4 x min spacing^2)
    d_max: float = 0.0                # depth clamp for probe rays (1.5 x cell diagonal)
    texel: str = "f32"                # texel storage: "f32" or "f16" (IEEE binary16)

    @property
    def count(self) -> int:
        return int(self.dims[0] * self.dims[1] * self.dims[2])


@dataclasses.dataclass
class Params:
    """Resampling parameters; one field per free constant of the method."""
    M: int = 32                       # initial candidates per pixel
    k: int = 5                        # spatial neighbours per pass
    n_spatial: int = 2                # spatial passes
    radius: float = 30.0              # spatial radius (pixels)
    g_max: float = 1.0                # geometry-term bound (Sec. 3.5)
    cos_n: float = math.cos(math.radians(25.0))   # reuse normal test
    depth_rel: float = 0.1            # reuse relative depth test
    m_cap: int = 20                   # temporal history cap, multiple of the current M
    unbiased: int = 1                 # 1: 1/Z normalisation with visibility, 0: 1/M
    temporal: bool = True
    M_light: int = 0                  # emitter-sampled candidates per pixel (M + M_light <= 32)
    subsample: int = 1                # n: pixel (x, y) draws candidates in frame f iff (x + y + f) % n == 0
    foot_c: float = 0.2               # footprint threshold c of the glossy shading recursion (Eq. 8)
    glossy_depth: int = 8             # most glossy vertices the shading recursion visits


@dataclasses.dataclass
class ProbeUpdate:
    rays: int = 256                   # rays per probe per pass
    hysteresis: float = 0.97
    sharpness: float = 50.0           # depth-moment cosine exponent
    fill_passes: int = 4              # passes at hysteresis 0 before frame 0
    fill_rays: int = 256
    per_frame: bool = False           # update every frame (4K workload)
    distance_slider: float = 0.0      # weight of the backward distance in the emission heuristic (0: off)


@dataclasses.dataclass
class Config:
    name: str
    width: int
    height: int
    scene_seed: int
    n_spheres: int
    n_boxes: int
    n_emitters: int
    room_lo: tuple
    room_hi: tuple
    size_lo: float
    size_hi: float
    emit_lo: float
    emit_hi: float
    eye: tuple
    look: tuple
    vfov_deg: float
    pan: float                        # camera translation along its right vector per frame
    probe_dims: tuple
    probe_spacing: float
    params: Params
    probe_update: ProbeUpdate
    frames: int
    grid_res: tuple                   # uniform-grid accelerator resolution
    seeds: tuple = (1, 2, 3)
    clear_emitters: bool = False      # redraw primitives that reach into an emitter
    glossy_frac: float = 0.0          # fraction of non-emitting primitives with a GGX specular layer
    spec_range: tuple = (0.3, 0.7)    # its weight ks, uniform (diffuse albedo scaled by 1 - ks)
    rough_range: tuple = (0.02, 0.5)  # its roughness alpha, log-uniform
    probe_texel: str = "f32"          # probe texel storage: "f32" (the workloads) or "f16"


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
CONFIGS = {
    # 64x64, room [0,8]^3 with 8 spheres, one of them an emitter of radiance 20;
    # 4x4x4 probes filled by 64 rays each; M=8, no temporal reuse, one spatial pass k=3.
    "tiny": Config(
        name="tiny", width=64, height=64, scene_seed=101, n_spheres=8, n_boxes=0,
        n_emitters=1, room_lo=(0, 0, 0), room_hi=(8, 8, 8), size_lo=0.3, size_hi=1.2,
        emit_lo=20.0, emit_hi=20.0, eye=(4, 4, 0.5), look=(4, 3.5, 8), vfov_deg=60.0,
        pan=0.0, probe_dims=(4, 4, 4), probe_spacing=2.0,
        params=Params(M=8, k=3, n_spatial=1, radius=8.0, temporal=False),
        probe_update=ProbeUpdate(rays=64, hysteresis=0.0, fill_passes=4, fill_rays=64),
        frames=1, grid_res=(8, 8, 8)),
    # 1920x1080, room [0,32]x[0,8]x[0,32] with 128 spheres + 128 boxes, 4 emitters;
    # 32x8x32 probes; M=32, temporal reuse, two spatial passes k=5 radius 30 px.
    "hd": Config(
        name="hd", width=1920, height=1080, scene_seed=102, n_spheres=128, n_boxes=128,
        n_emitters=4, room_lo=(0, 0, 0), room_hi=(32, 8, 32), size_lo=0.2, size_hi=1.5,
        emit_lo=10.0, emit_hi=50.0, eye=(16, 4, 1), look=(16, 3, 31), vfov_deg=60.0,
        pan=0.05, probe_dims=(32, 8, 32), probe_spacing=1.0,
        params=Params(M=32, k=5, n_spatial=2, radius=30.0, temporal=True),
        probe_update=ProbeUpdate(rays=256, hysteresis=0.0, fill_passes=4, fill_rays=256),
        frames=8, grid_res=(12, 3, 12)),
    # 3840x2160, same room with 512 + 512 primitives, 64x16x64 probes updated every
    # frame with 256 rays at hysteresis 0.97.  Four times the primitives of the
    # 1920x1080 room at the same occupancy (sizes scaled by 4^(-1/3)) and with
    # the same emitters per primitive (16), none of them reached into.
    "uhd": Config(
        name="uhd", width=3840, height=2160, scene_seed=103, n_spheres=512, n_boxes=512,
        n_emitters=16, room_lo=(0, 0, 0), room_hi=(32, 8, 32), size_lo=0.125, size_hi=0.95,
        emit_lo=10.0, emit_hi=50.0, eye=(16, 4, 1), look=(16, 3, 31), vfov_deg=60.0,
        pan=0.05, probe_dims=(64, 16, 64), probe_spacing=0.5,
        params=Params(M=32, k=5, n_spatial=2, radius=30.0, temporal=True),
        probe_update=ProbeUpdate(rays=256, hysteresis=0.97, fill_passes=4, fill_rays=256,
                                 per_frame=True),
        frames=16, grid_res=(24, 6, 24), clear_emitters=True),
    # Glossy workloads (the glossy L_DDGI+ and the specular recursion): the
    # tiny room with four boxes added, and the 1920x1080 room, with 60% / 50%
    # of the non-emitting primitives given a GGX specular layer, ks
    # U[0.3, 0.7], roughness log-uniform in [0.02, 0.5].
    "glossy_tiny": Config(
        name="glossy_tiny", width=64, height=64, scene_seed=111, n_spheres=8, n_boxes=4,
        n_emitters=1, room_lo=(0, 0, 0), room_hi=(8, 8, 8), size_lo=0.3, size_hi=1.2,
        emit_lo=20.0, emit_hi=20.0, eye=(4, 4, 0.5), look=(4, 3.5, 8), vfov_deg=60.0,
        pan=0.0, probe_dims=(4, 4, 4), probe_spacing=2.0,
        params=Params(M=8, k=3, n_spatial=1, radius=8.0, temporal=False),
        probe_update=ProbeUpdate(rays=64, hysteresis=0.0, fill_passes=4, fill_rays=64),
        frames=1, grid_res=(8, 8, 8), glossy_frac=0.6),
    "glossy": Config(
        name="glossy", width=1920, height=1080, scene_seed=102, n_spheres=128, n_boxes=128,
        n_emitters=4, room_lo=(0, 0, 0), room_hi=(32, 8, 32), size_lo=0.2, size_hi=1.5,
        emit_lo=10.0, emit_hi=50.0, eye=(16, 4, 1), look=(16, 3, 31), vfov_deg=60.0,
        pan=0.05, probe_dims=(32, 8, 32), probe_spacing=1.0,
        params=Params(M=32, k=5, n_spatial=2, radius=30.0, temporal=True),
        probe_update=ProbeUpdate(rays=256, hysteresis=0.0, fill_passes=4, fill_rays=256),
        frames=8, grid_res=(12, 3, 12), glossy_frac=0.5),
}


def _camera_basis(eye, look):
    eye = np.asarray(eye, np.float64)
    f = np.asarray(look, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.array([0.0, 1.0, 0.0]))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return eye, f, r, u


def make_camera(cfg: Config, frame: int = 0, width: Optional[int] = None,
                height: Optional[int] = None) -> Camera:
    eye, f, r, u = _camera_basis(cfg.eye, cfg.look)
    eye = eye + cfg.pan * frame * r
    return Camera(eye=eye.astype(np.float32), fwd=f.astype(np.float32),
                  right=r.astype(np.float32), up=u.astype(np.float32),
                  tan_half_fovy=float(np.float32(math.tan(math.radians(cfg.vfov_deg) / 2))),
                  width=int(width or cfg.width), height=int(height or cfg.height))


def _dist_point_segment(p, a, b):
    ab = b - a
    t = np.clip(np.dot(p - a, ab) / max(np.dot(ab, ab), 1e-12), 0.0, 1.0)
    return np.linalg.norm(p - (a + t * ab))


def make_scene(cfg: Config, max_frames: int = 32) -> Scene:
    """Seeded room: spheres first (the first n_emitters of them emit), then boxes.
    Primitives that would swallow the camera path (all frames up to max_frames)
    are redrawn, so the eye is never inside geometry; with clear_emitters,
    so are primitives whose bounding sphere reaches into an emitter's, so no
    light is enclosed."""
    rng = np.random.default_rng(cfg.scene_seed)
    lo = np.asarray(cfg.room_lo, np.float64)
    hi = np.asarray(cfg.room_hi, np.float64)
    eye, _, r, _ = _camera_basis(cfg.eye, cfg.look)
    a, b = eye, eye + cfg.pan * max_frames * r
    types, centers, sizes, albedo, emit = [], [], [], [], []
    lights = []                                    # (centre, radius) of the emitters drawn so far
    for i in range(cfg.n_spheres + cfg.n_boxes):
        is_sphere = i < cfg.n_spheres
        while True:
            if is_sphere:
                rad = rng.uniform(cfg.size_lo, cfg.size_hi)
                half = np.array([rad, rad, rad])
            else:
                half = rng.uniform(cfg.size_lo, cfg.size_hi, 3)
            c = rng.uniform(lo + half, hi - half)
            reach = np.linalg.norm(half) if not is_sphere else half[0]
            clear = not cfg.clear_emitters or all(
                np.linalg.norm(c - ec) > reach + er for ec, er in lights)
            if _dist_point_segment(c, a, b) > reach + 0.3 and clear:
                break
        types.append(PRIM_SPHERE if is_sphere else PRIM_BOX)
        centers.append(c)
        sizes.append([half[0], 0.0, 0.0] if is_sphere else half)
        if is_sphere and i < cfg.n_emitters:
            albedo.append([0.0, 0.0, 0.0])
            le = rng.uniform(cfg.emit_lo, cfg.emit_hi)
            emit.append([le, le, le])
            lights.append((c, half[0]))
        else:
            albedo.append(rng.uniform(0.1, 0.9, 3))
            emit.append([0.0, 0.0, 0.0])
    spec = rough = None
    if cfg.glossy_frac > 0.0:
        # the specular layers come from a stream of their own, so the geometry
        # and albedo draws are those of the same room without them
        grng = np.random.default_rng(cfg.scene_seed + 7919)
        spec, rough = np.zeros(len(types)), np.ones(len(types))
        for i in range(len(types)):
            has = grng.random() < cfg.glossy_frac
            ks = grng.uniform(*cfg.spec_range)
            al = float(np.exp(grng.uniform(np.log(cfg.rough_range[0]), np.log(cfg.rough_range[1]))))
            if has and not np.any(np.asarray(emit[i]) > 0):
                spec[i], rough[i] = ks, al
                albedo[i] = np.asarray(albedo[i]) * (1.0 - ks)
    prims = prim_records(types, centers, sizes, albedo, emit, spec, rough)
    ext = float(np.max(hi - lo))
    return Scene(prims=prims, has_room=True, room_lo=lo.astype(np.float32),
                 room_hi=hi.astype(np.float32),
                 wall_albedo=np.full(3, 0.8, np.float32), sky=np.zeros(3, np.float32),
                 eps=float(np.float32(1e-4 * ext)))


def make_probe_grid(cfg: Config) -> ProbeGrid:
    s = float(cfg.probe_spacing)
    return probe_grid(cfg.probe_dims, cfg.room_lo, s, texel=cfg.probe_texel)


def probe_grid(dims, lo, spacing, irr_res=8, dep_res=16, texel="f32") -> ProbeGrid:
    s = float(spacing)
    return ProbeGrid(dims=tuple(int(v) for v in dims),
                     lo=np.asarray(lo, np.float32).reshape(3),
                     spacing=np.full(3, s, np.float32), irr_res=irr_res, dep_res=dep_res,
                     bias_dist=float(np.float32(0.3 * s)),
                     var_floor=float(np.float32(1e-4 * s * s)),
                     d_max=float(np.float32(1.5 * s * math.sqrt(3.0))), texel=texel)


def empty_probe_textures(grid: ProbeGrid):
    """Zero irradiance (RGBA f32, alpha unused) and zero depth moments (f32 x2),
    gutter-padded: (P, (N+2)^2, 4) and (P, (Nd+2)^2, 2)."""
    P = grid.count
    irr = np.zeros((P, (grid.irr_res + 2) ** 2, 4), np.float32)
    dep = np.zeros((P, (grid.dep_res + 2) ** 2, 2), np.float32)
    return irr, dep


def random_probe_textures(grid: ProbeGrid, seed: int):
    """Seeded stand-in probe textures for parity tests at full size (both
    sides read the same arrays): irradiance texels U[0, 2), depth means
    U[0.05, d_max) with second moments mean^2 + U[0, 0.05) spacing^2.
    Plain random numbers, gutters included."""
    rng = np.random.default_rng(seed)
    P = grid.count
    irr = np.zeros((P, (grid.irr_res + 2) ** 2, 4), np.float32)
    irr[..., :3] = rng.uniform(0.0, 2.0, (P, (grid.irr_res + 2) ** 2, 3))
    dep = np.zeros((P, (grid.dep_res + 2) ** 2, 2), np.float32)
    m = rng.uniform(0.05, grid.d_max, (P, (grid.dep_res + 2) ** 2))
    s = float(min(grid.spacing))
    dep[..., 0] = m
    dep[..., 1] = m * m + rng.uniform(0.0, 0.05, m.shape) * s * s
    return irr, dep


# --------------------------------------------------------------------------
# closed-form test scenes
# --------------------------------------------------------------------------
def furnace_plane(albedo=(0.5, 0.7, 0.9), sky=(1.0, 2.0, 3.0), size=1000.0) -> Scene:
    """A very large Lambertian slab whose top face is y=0, under a uniform sky."""
    prims = prim_records([PRIM_BOX], [[0.0, -1.0, 0.0]], [[size, 1.0, size]],
                         [albedo], [[0.0, 0.0, 0.0]])
    return Scene(prims=prims, has_room=False, room_lo=np.zeros(3, np.float32),
                 room_hi=np.zeros(3, np.float32), wall_albedo=np.zeros(3, np.float32),
                 sky=np.asarray(sky, np.float32), eps=float(np.float32(1e-3)))


def furnace_camera(width=32, height=32, height_above=2.0) -> Camera:
    eye = np.array([0.0, height_above, 0.0])
    look = np.array([0.3, 0.0, 4.0])
    f = look - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, [0.0, 1.0, 0.0])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return Camera(eye=eye.astype(np.float32), fwd=f.astype(np.float32),
                  right=r.astype(np.float32), up=u.astype(np.float32),
                  tan_half_fovy=float(np.float32(math.tan(math.radians(30.0)))),
                  width=width, height=height)


def emissive_room_sphere(albedo=(0.3, 0.6, 0.9), radiance=(2.0, 1.0, 0.5)) -> Scene:
    """A convex sphere in the middle of a room whose walls emit `radiance` and
    reflect nothing: every point of the sphere sees only walls."""
    prims = prim_records([PRIM_SPHERE], [[4.0, 4.0, 4.0]], [[1.0, 0.0, 0.0]],
                         [albedo], [[0.0, 0.0, 0.0]])
    return Scene(prims=prims, has_room=True, room_lo=np.zeros(3, np.float32),
                 room_hi=np.full(3, 8.0, np.float32), wall_albedo=np.zeros(3, np.float32),
                 sky=np.zeros(3, np.float32), eps=float(np.float32(8e-4)),
                 wall_emit=np.asarray(radiance, np.float32))


def shadow_scene() -> Scene:
    """Floor slab (top at y=0), an emissive sphere above it and a wall that
    casts a sharp shadow across the floor; black sky.  Neighbouring pixels
    on the two sides of the shadow edge disagree on the emitter's visibility."""
    prims = prim_records(
        [PRIM_BOX, PRIM_SPHERE, PRIM_BOX],
        [[0.0, -1.0, 0.0], [0.0, 3.0, -1.0], [0.0, 0.5, 0.0]],
        [[50.0, 1.0, 50.0], [0.4, 0.0, 0.0], [3.0, 0.5, 0.05]],
        [[0.6, 0.6, 0.6], [0.0, 0.0, 0.0], [0.5, 0.5, 0.5]],
        [[0.0, 0.0, 0.0], [20.0, 20.0, 20.0], [0.0, 0.0, 0.0]])
    return Scene(prims=prims, has_room=False, room_lo=np.zeros(3, np.float32),
                 room_hi=np.zeros(3, np.float32), wall_albedo=np.zeros(3, np.float32),
                 sky=np.zeros(3, np.float32), eps=float(np.float32(1e-3)))


def shadow_camera(width=16, height=16) -> Camera:
    eye = np.array([0.0, 4.0, 2.5])
    look = np.array([0.0, 0.0, 0.6])
    f = look - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, [0.0, 1.0, 0.0])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return Camera(eye=eye.astype(np.float32), fwd=f.astype(np.float32),
                  right=r.astype(np.float32), up=u.astype(np.float32),
                  tan_half_fovy=float(np.float32(math.tan(math.radians(15.0)))),
                  width=width, height=height)
