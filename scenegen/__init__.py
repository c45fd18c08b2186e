"""Seeded synthetic inputs for the hybrid depth-of-field path.

This module builds scenes, cameras, lenses, lights and camera paths from a
seed.  It holds none of the method's arithmetic (no ray generation, no
circle of confusion, no filtering): it only produces the triangle soups and
the camera/lens parameters that both the GPU library and the FP64 oracle
consume.  Every array it returns is float32, the precision of the library's
interface, so that the oracle widens exactly the same values.

Scene shapes stand in for the paper's indoor close-up (a foreground cushion
partly covering a background cushion, Fig. 1), which is not available.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np

F32 = np.float32


@dataclass
class Camera:
    """Pinhole frame of the thin-lens camera: eye, orthonormal right/up/forward,
    tan of the horizontal half field of view, image size in pixels."""
    eye: np.ndarray
    right: np.ndarray
    up: np.ndarray
    fwd: np.ndarray
    tan_half_fov_x: float
    width: int
    height: int

    def as_floats(self) -> np.ndarray:
        """13 float32 values: eye, right, up, fwd, tan_half_fov_x."""
        return np.concatenate([self.eye, self.right, self.up, self.fwd,
                               [self.tan_half_fov_x]]).astype(F32)


@dataclass
class Lens:
    """Thin lens: focal length f (m), aperture diameter A = f/N (m), focus
    distance S1 (m); aperture shape: blades = 0 (a disk) or a regular
    polygon of that many blades (>= 3) inscribed in the disk, rotated by
    `rotation` (rad); spherical aberration `sa` (relative sample weight
    1 + sa (2 rho^2 - 1) at normalised radius rho, clamped at 0)."""
    focal_length: float
    aperture: float
    focus_distance: float
    blades: int = 0
    rotation: float = 0.0
    sa: float = 0.0

    def as_floats(self) -> np.ndarray:
        return np.array([self.focal_length, self.aperture, self.focus_distance, self.blades, self.rotation,
                         self.sa], F32)


@dataclass
class Light:
    """One point light with rgb intensity plus an rgb ambient term."""
    pos: np.ndarray
    intensity: np.ndarray
    ambient: np.ndarray

    def as_floats(self) -> np.ndarray:
        return np.concatenate([self.pos, self.intensity, self.ambient]).astype(F32)


@dataclass
class Scene:
    verts: np.ndarray   # (n, 9) float32: v0.xyz, v1.xyz, v2.xyz
    albedo: np.ndarray  # (n, 3) float32
    meta: dict = field(default_factory=dict)
    spec: np.ndarray | None = None  # (n, 2) float32 (k_s, shininess) or None: Lambertian

    @property
    def n_tris(self) -> int:
        return int(self.verts.shape[0])


@dataclass
class MaskParams:
    sigma: float = 1.0
    tau_depth: float = 0.05
    tau_normal: float = 0.1
    tau_var: float = 0.01
    var_alpha: float = 0.2
    spp_max: int = 8
    tile: int = 8
    dilate: int = 1


@dataclass
class PPParams:
    n_taps: int = 48
    tile: int = 16
    r_cap: float = 64.0
    bg_ramp_px: float = 1.0


@dataclass
class CompositeParams:
    h_t: float = 0.5
    rt_override: int = 0
    spec_y: float = 0.0  # > 0: specular luminance at which near traced pixels take the post-process colour


@dataclass
class ReconParams:
    enable: bool = False
    alpha: float = 0.2


@dataclass
class SpatialParams:
    enable: bool = False
    n_taps: int = 24
    r_cap: float = 64.0
    v_clamp: float = 0.01


@dataclass
class FrameConfig:
    """Everything one frame of the path needs besides the scene."""
    name: str
    camera: Camera
    lens: Lens
    light: Light
    mask: MaskParams
    pp: PPParams
    comp: CompositeParams
    seed: int = 0
    recon: ReconParams = field(default_factory=ReconParams)
    spatial: SpatialParams = field(default_factory=SpatialParams)


# ----------------------------------------------------------------------------
# camera helpers
# ----------------------------------------------------------------------------

def look_camera(eye, yaw_deg: float, width: int, height: int,
                tan_half_fov_x: float = 0.36) -> Camera:
    """Camera at `eye` looking along +z rotated by `yaw_deg` about +y, y up."""
    psi = math.radians(yaw_deg)
    fwd = np.array([math.sin(psi), 0.0, math.cos(psi)])
    right = np.array([math.cos(psi), 0.0, -math.sin(psi)])
    up = np.array([0.0, 1.0, 0.0])
    return Camera(np.asarray(eye, F32), right.astype(F32), up.astype(F32),
                  fwd.astype(F32), float(F32(tan_half_fov_x)), int(width), int(height))


def lens_fnumber(f: float, n: float, focus: float) -> Lens:
    return Lens(float(F32(f)), float(F32(f / n)), float(F32(focus)))


# ----------------------------------------------------------------------------
# geometry builders (triangle soups)
# ----------------------------------------------------------------------------

def _quad(a, b, c, d):
    """Two triangles (a, b, c) and (a, c, d)."""
    return [np.concatenate([a, b, c]), np.concatenate([a, c, d])]


def room_box(lo, hi) -> np.ndarray:
    """Closed axis-aligned box, 12 triangles."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    p = [np.array(v, np.float64) for v in [
        (x0, y0, z0), (x1, y0, z0), (x1, y1, z0), (x0, y1, z0),
        (x0, y0, z1), (x1, y0, z1), (x1, y1, z1), (x0, y1, z1)]]
    faces = [(0, 1, 2, 3), (5, 4, 7, 6), (4, 0, 3, 7), (1, 5, 6, 2),
             (4, 5, 1, 0), (3, 2, 6, 7)]
    tris = []
    for a, b, c, d in faces:
        tris += _quad(p[a], p[b], p[c], p[d])
    return np.stack(tris)


def grid_box(center, half, n: int) -> np.ndarray:
    """Axis-aligned cube with each face tessellated into an n x n grid
    (6 n^2 quads, 12 n^2 triangles)."""
    c = np.asarray(center, np.float64)
    t = np.linspace(-1.0, 1.0, n + 1)
    tris = []
    for axis in range(3):
        a1, a2 = (axis + 1) % 3, (axis + 2) % 3
        for side in (-1.0, 1.0):
            g = np.zeros((n + 1, n + 1, 3))
            g[..., axis] = side
            g[..., a1] = t[:, None]
            g[..., a2] = t[None, :]
            g = c + half * g
            v00 = g[:-1, :-1].reshape(-1, 3)
            v10 = g[1:, :-1].reshape(-1, 3)
            v11 = g[1:, 1:].reshape(-1, 3)
            v01 = g[:-1, 1:].reshape(-1, 3)
            tris.append(np.concatenate([v00, v10, v11], 1))
            tris.append(np.concatenate([v00, v11, v01], 1))
    return np.concatenate(tris)


def uv_sphere(center, radius, stacks: int, slices: int) -> np.ndarray:
    """UV sphere: 2*slices cap triangles + 2*slices*(stacks-2) band triangles."""
    c = np.asarray(center, np.float64)
    th = np.linspace(0.0, math.pi, stacks + 1)
    ph = np.linspace(0.0, 2 * math.pi, slices + 1)
    st, ct = np.sin(th), np.cos(th)
    sp, cp = np.sin(ph), np.cos(ph)
    P = np.stack([st[:, None] * cp[None, :], ct[:, None] * np.ones_like(ph)[None, :],
                  st[:, None] * sp[None, :]], -1) * radius + c
    tris = []
    for i in range(stacks):
        a = P[i, :-1]
        b = P[i + 1, :-1]
        cc = P[i + 1, 1:]
        d = P[i, 1:]
        if i != stacks - 1:
            tris.append(np.concatenate([a, b, cc], 1))
        if i != 0:
            tris.append(np.concatenate([a, cc, d], 1))
    return np.concatenate(tris)


WALL_ALBEDO = (0.8, 0.75, 0.7)


def _assemble(parts, albedos, meta) -> Scene:
    verts = np.concatenate(parts).astype(F32)
    alb = np.concatenate([np.broadcast_to(np.asarray(a, np.float64), (p.shape[0], 3))
                          if np.ndim(a) == 1 else a for p, a in zip(parts, albedos)])
    meta = dict(meta, part_tris=[int(p.shape[0]) for p in parts])
    return Scene(np.ascontiguousarray(verts), np.ascontiguousarray(alb.astype(F32)), meta)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def tiny_scene(seed: int = 0, n_random: int = 256) -> Scene:
    """64x64 workload scene: room box [-2,2]x[-2,2]x[-1,6] + random triangles
    with x, y ~ U[-1, 1] and z ~ U[1, 4] per vertex, albedo U[0,1]^3."""
    rng = np.random.default_rng(seed)
    room = room_box((-2, -2, -1), (2, 2, 6))
    xy = rng.uniform(-1.0, 1.0, (n_random, 3, 2))
    z = rng.uniform(1.0, 4.0, (n_random, 3, 1))
    rnd = np.concatenate([xy, z], -1).reshape(n_random, 9)
    alb = rng.uniform(0.0, 1.0, (n_random, 3))
    return _assemble([room, rnd], [WALL_ALBEDO, alb], {"name": "tiny", "seed": seed})


def living_room_scene(seed: int = 0, n_objects: int = 20, depth_max: float = 6.0,
                      room_far: float = 7.0, sphere_res=(70, 72), box_res: int = 29,
                      tan_half_fov_x: float = 0.36, aspect: float = 1080 / 1920) -> Scene:
    """Procedural living room: room box, two fixed box 'cushions' (a small one
    at 0.6 m partly covering a large one at 2.5 m), and random tessellated
    spheres and boxes at axial depth U[1.2, depth_max] inside 90 % of the
    view frustum, size U[0.15, 0.5] m, albedo U[0,1]^3, kept at least 0.8 m
    from the camera so the cushions stay visible.  Half the objects are
    spheres and half boxes."""
    rng = np.random.default_rng(seed)
    room = room_box((-3.0, -1.2, -0.5), (3.0, 1.8, room_far))
    parts, albs = [room], [WALL_ALBEDO]
    kinds = []
    # fixed cushions (boxes)
    fixed = [((0.072, -0.036, 0.6), 0.1), ((0.125, 0.05, 2.5), 0.3)]
    for cen, half in fixed:
        parts.append(grid_box(cen, half, box_res))
        albs.append(rng.uniform(0.0, 1.0, 3))
        kinds.append("box")
    n_rest = n_objects - len(fixed)
    n_sph = n_objects // 2
    for i in range(n_rest):
        size = rng.uniform(0.15, 0.5)
        z = rng.uniform(max(1.2, size + 0.8), depth_max)
        tx = tan_half_fov_x
        ty = tan_half_fov_x * aspect
        x = rng.uniform(-0.9, 0.9) * tx * z
        y = rng.uniform(-0.9, 0.9) * ty * z
        alb = rng.uniform(0.0, 1.0, 3)
        if i < n_sph:
            parts.append(uv_sphere((x, y, z), size, *sphere_res))
            kinds.append("sphere")
        else:
            parts.append(grid_box((x, y, z), size, box_res))
            kinds.append("box")
        albs.append(alb)
    return _assemble(parts, albs, {"name": "living_room", "seed": seed,
                                   "n_objects": n_objects, "kinds": kinds})


def glossy_living_room_scene(seed: int = 0, **kw) -> Scene:
    """The living room with specular materials: every object gets a
    Blinn-Phong lobe with k_s ~ U[0.3, 1], shininess ~ U[16, 256] for the
    spheres and U[4, 32] for the boxes (broad highlights on flat faces);
    the walls stay Lambertian.  These are the highlights whose bokeh the
    composite treats apart."""
    sc = living_room_scene(seed, **kw)
    rng = np.random.default_rng(seed + 1000)
    spec = np.zeros((sc.n_tris, 2), F32)
    spec[:, 1] = 1.0
    counts = sc.meta["part_tris"]
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    for kind, a, n in zip(["room"] + sc.meta["kinds"], starts, counts):
        if kind == "room":
            continue
        spec[a:a + n, 0] = rng.uniform(0.3, 1.0)
        spec[a:a + n, 1] = rng.uniform(16.0, 256.0) if kind == "sphere" else rng.uniform(4.0, 32.0)
    sc.spec = spec
    sc.meta = dict(sc.meta, name="glossy_living_room")
    return sc


def default_light_tiny() -> Light:
    return Light(np.array([0.0, 1.5, 1.0], F32), np.full(3, 4.0, F32), np.full(3, 0.05, F32))


def default_light_room() -> Light:
    return Light(np.array([0.6, 1.5, 0.2], F32), np.full(3, 6.0, F32), np.full(3, 0.05, F32))


def config_tiny(aperture_override: float | None = None) -> FrameConfig:
    """64x64, f = 50 mm, f/2, focus 2 m, 1-4 spp, seed 0."""
    cam = look_camera((0, 0, 0), 0.0, 64, 64)
    lens = lens_fnumber(0.05, 2.0, 2.0)
    if aperture_override is not None:
        lens = replace(lens, aperture=float(F32(aperture_override)))
    return FrameConfig("tiny" if aperture_override is None else "tiny_strong", cam, lens,
                       default_light_tiny(), MaskParams(spp_max=4), PPParams(), CompositeParams(), 0)


def config_1080p(width: int = 1920, height: int = 1080) -> FrameConfig:
    """1920x1080, f = 50 mm, f/1.4, focus 2 m, Gaussian sigma 1, 0-8 spp."""
    cam = look_camera((0, 0, 0), 0.0, width, height)
    lens = lens_fnumber(0.05, 1.4, 2.0)
    return FrameConfig("living_room_1080p", cam, lens, default_light_room(),
                       MaskParams(spp_max=8), PPParams(), CompositeParams(), 0)


def temporal_scene(seed: int = 1) -> Scene:
    """~1M-triangle variant: 100 objects at depth 0.5-8 m, room to z = 9 m."""
    return living_room_scene(seed, n_objects=100, depth_max=8.0, room_far=9.0)


def temporal_camera(t: int, width: int = 1920, height: int = 1080) -> Camera:
    """Dolly 1 cm per frame along +z with 0.2 degree yaw per frame."""
    return look_camera((0.0, 0.0, 0.01 * t), 0.2 * t, width, height)


def config_temporal(width: int = 1920, height: int = 1080) -> FrameConfig:
    cam = temporal_camera(0, width, height)
    lens = lens_fnumber(0.05, 1.4, 1.5)
    return FrameConfig("temporal_1080p", cam, lens, default_light_room(),
                       MaskParams(spp_max=16, var_alpha=0.2), PPParams(), CompositeParams(), 0)


BATCH_RESOLUTIONS = [(640, 360), (1280, 720), (1920, 1080), (2560, 1440)]


def batched_views(seed: int = 7, n_views: int = 32):
    """Views of the 1080p scene: resolution uniform over four sizes, focus
    U[0.8, 5] m, f-number in {1.4, 2, 2.8}, eye offset U[-0.2, 0.2] m in x and
    y, yaw U[-10, 10] degrees."""
    rng = np.random.default_rng(seed)
    out = []
    for v in range(n_views):
        w, h = BATCH_RESOLUTIONS[int(rng.integers(0, 4))]
        s1 = rng.uniform(0.8, 5.0)
        n = [1.4, 2.0, 2.8][int(rng.integers(0, 3))]
        ex, ey = rng.uniform(-0.2, 0.2, 2)
        yaw = rng.uniform(-10.0, 10.0)
        cam = look_camera((ex, ey, 0.0), yaw, w, h)
        lens = lens_fnumber(0.05, n, s1)
        out.append(FrameConfig(f"view{v}", cam, lens, default_light_room(),
                               MaskParams(spp_max=8), PPParams(), CompositeParams(), seed))
    return out


def half_plane_scene(z_near: float, x_edge: float, z_far: float) -> Scene:
    """A large near occluder covering x < x_edge at depth z_near over a far wall
    at depth z_far.  Used for the partial-occlusion hit-ratio pin."""
    big = 50.0
    occ = np.array([[-big, -big, z_near, x_edge, -big, z_near, x_edge, big, z_near],
                    [-big, -big, z_near, x_edge, big, z_near, -big, big, z_near]])
    wall = np.array([[-big, -big, z_far, big, -big, z_far, big, big, z_far],
                     [-big, -big, z_far, big, big, z_far, -big, big, z_far]])
    return _assemble([occ, wall], [(1.0, 0.0, 0.0), (0.0, 0.0, 1.0)], {"name": "half_plane"})


def spatial_inputs(H: int, W: int, seed: int, coverage: float, coc_max: float = 150.0) -> dict:
    """Seeded per-pixel inputs of the spatial reconstruction shaped like a
    frame's: traced pixels clustered in 8x8 tiles (a fraction `coverage` of
    the tiles, 90 % of their pixels, 1-8 rays each), hit ratios with mass at
    0 and 1, colours in [0, 1.5], near/far CoC sizes in [0, coc_max] px,
    accumulated hit ratios, and variance estimates in [0, 0.03] with 10 %
    not yet estimated (+inf)."""
    rng = np.random.default_rng(seed)
    TH, TW = -(-H // 8), -(-W // 8)
    tiles = rng.uniform(size=(TH, TW)) < coverage
    on = np.repeat(np.repeat(tiles, 8, 0), 8, 1)[:H, :W] & (rng.uniform(size=(H, W)) < 0.9)
    spp = np.where(on, rng.integers(1, 9, (H, W)), 0).astype(np.uint8)
    h = rng.uniform(0, 1, (H, W))
    u = rng.uniform(size=(H, W))
    h[u < 0.3] = 1.0
    h[(u >= 0.3) & (u < 0.45)] = 0.0
    V = rng.uniform(0, 0.03, (H, W))
    V[rng.uniform(size=(H, W)) < 0.1] = np.inf
    return dict(spp=spp,
                c_near=rng.uniform(0, 1.5, (3, H, W)).astype(F32),
                c_far=rng.uniform(0, 1.5, (3, H, W)).astype(F32),
                hit_ratio=h.astype(F32),
                hit_acc=rng.uniform(0, 1, (H, W)).astype(F32),
                coc_nf=rng.uniform(0, coc_max, (2, H, W)).astype(F32),
                variance=V.astype(F32))


def random_rgb(shape, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 1.0, shape).astype(F32)
