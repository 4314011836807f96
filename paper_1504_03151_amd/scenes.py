"""Seeded synthetic scenes, cameras and render settings.

This module only *generates inputs*: sphere lists, triangle meshes, planes,
materials, lights, cameras and render parameters, all drawn from
``numpy.random.default_rng(seed)``.  It contains none of the ray tracer's
arithmetic (no intersection, no shading), so the GPU path and the FP64 oracle
can both consume its output without sharing any of the method.

Geometry is stored in FP32 (the library's input format); the oracle widens the
same values exactly to FP64.

Material rows are ``[albedo_r, albedo_g, albedo_b, k_a, k_d, k_s, shininess,
k_r, ior, type]`` with ``type`` 0 = Phong, 1 = mirror, 2 = dielectric.  Lights
are ``[x, y, z, I_r, I_g, I_b, shape, u_x, u_y, u_z, v_x, v_y, v_z]``: shape 0
a point light at (x, y, z), 1 the parallelogram spanned by u and v from it, 2
the ellipse (a disk when u and v are orthogonal and of equal length) centred
on it; six-column rows are point lights.

The scene recipes stand in for the paper's sphere scene (Section V, 640x480,
not distributed): a small random-sphere scene, a large heightfield terrain with
mirror spheres, a large icosphere field with mixed materials, a batch of uneven
scenes, and the same icosphere field for the learned radiance cache.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

PHONG, MIRROR, DIELECTRIC = 0, 1, 2
MAT_COLS = 10
LIGHT_COLS = 13
POINT, PARALLELOGRAM, DISK = 0, 1, 2


@dataclasses.dataclass
class Scene:
    spheres: np.ndarray      # (ns, 4) f32: cx, cy, cz, r
    sphere_mat: np.ndarray   # (ns,) i32
    tris: np.ndarray         # (nt, 3, 3) f32: CCW seen from outside
    tri_mat: np.ndarray      # (nt,) i32
    planes: np.ndarray       # (np, 4) f32: nx, ny, nz, h  (n . x = h, |n| = 1)
    plane_mat: np.ndarray    # (np,) i32
    materials: np.ndarray    # (nm, 10) f32
    lights: np.ndarray       # (nl, 13) f32: pos, intensity, shape, u, v
    name: str = "scene"

    @property
    def n_prims(self) -> int:
        return len(self.spheres) + len(self.tris) + len(self.planes)

    def validate_shapes(self) -> None:
        assert self.spheres.dtype == np.float32 and self.spheres.ndim == 2 and self.spheres.shape[1] == 4
        assert self.tris.dtype == np.float32 and self.tris.ndim == 3 and self.tris.shape[1:] == (3, 3)
        assert self.planes.dtype == np.float32 and self.planes.ndim == 2 and self.planes.shape[1] == 4
        assert self.materials.dtype == np.float32 and self.materials.shape[1] == MAT_COLS
        assert self.lights.dtype == np.float32 and self.lights.shape[1] == LIGHT_COLS
        assert len(self.sphere_mat) == len(self.spheres)
        assert len(self.tri_mat) == len(self.tris)
        assert len(self.plane_mat) == len(self.planes)


@dataclasses.dataclass
class Camera:
    eye: Tuple[float, float, float]
    look_at: Tuple[float, float, float]
    up: Tuple[float, float, float]
    vfov_deg: float
    width: int
    height: int

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Params:
    spp: int = 1
    max_depth: int = 3
    jitter: int = 0
    seed: int = 0
    frame: int = 0
    bg: Tuple[float, float, float] = (0.1, 0.2, 0.3)
    eps: float = 1e-3
    gi: int = 0          # 1: diffuse global illumination by path tracing


@dataclasses.dataclass
class Workload:
    scene: Scene
    camera: Camera
    params: Params
    name: str


def _empty_f32(*shape):
    return np.zeros(shape, dtype=np.float32)


def _empty_i32(n=0):
    return np.zeros((n,), dtype=np.int32)


def make_scene(spheres=None, sphere_mat=None, tris=None, tri_mat=None, planes=None,
               plane_mat=None, materials=None, lights=None, name="scene") -> Scene:
    sp = _empty_f32(0, 4) if spheres is None else np.ascontiguousarray(spheres, dtype=np.float32).reshape(-1, 4)
    tr = _empty_f32(0, 3, 3) if tris is None else np.ascontiguousarray(tris, dtype=np.float32).reshape(-1, 3, 3)
    pl = _empty_f32(0, 4) if planes is None else np.ascontiguousarray(planes, dtype=np.float32).reshape(-1, 4)
    sm = _empty_i32(len(sp)) if sphere_mat is None else np.ascontiguousarray(sphere_mat, dtype=np.int32).reshape(-1)
    tm = _empty_i32(len(tr)) if tri_mat is None else np.ascontiguousarray(tri_mat, dtype=np.int32).reshape(-1)
    pm = _empty_i32(len(pl)) if plane_mat is None else np.ascontiguousarray(plane_mat, dtype=np.int32).reshape(-1)
    mats = np.ascontiguousarray(materials, dtype=np.float32).reshape(-1, MAT_COLS)
    li = np.asarray(lights if lights is not None else np.zeros((0, 6)), dtype=np.float32)
    li = li.reshape(len(li), -1) if li.size else np.zeros((0, 6), np.float32)
    if li.shape[1] == 6:      # point lights
        li = np.hstack([li, np.zeros((len(li), LIGHT_COLS - 6), np.float32)])
    li = np.ascontiguousarray(li, dtype=np.float32).reshape(-1, LIGHT_COLS)
    s = Scene(sp, sm, tr, tm, pl, pm, mats, li, name)
    s.validate_shapes()
    return s


def material(albedo=(1.0, 1.0, 1.0), k_a=0.1, k_d=1.0, k_s=0.5, shininess=32.0, k_r=0.0,
             ior=1.5, mtype=PHONG) -> np.ndarray:
    return np.array([albedo[0], albedo[1], albedo[2], k_a, k_d, k_s, shininess, k_r, ior, mtype],
                    dtype=np.float32)


def mirror_material(k_r=0.9, k_s=0.5) -> np.ndarray:
    return material((1.0, 1.0, 1.0), k_a=0.0, k_d=0.0, k_s=k_s, k_r=k_r, mtype=MIRROR)


def dielectric_material(ior=1.5, k_s=0.5) -> np.ndarray:
    return material((1.0, 1.0, 1.0), k_a=0.0, k_d=0.0, k_s=k_s, k_r=0.0, ior=ior, mtype=DIELECTRIC)


# --------------------------------------------------------------------------
# Meshes
# --------------------------------------------------------------------------

def icosphere(subdivisions: int) -> np.ndarray:
    """Unit icosphere as (20 * 4**subdivisions, 3, 3) float64 triangles, CCW outward."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, g, 0), (1, g, 0), (-1, -g, 0), (1, -g, 0),
             (0, -1, g), (0, 1, g), (0, -1, -g), (0, 1, -g),
             (g, 0, -1), (g, 0, 1), (-g, 0, -1), (-g, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    v = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in verts]
    for _ in range(subdivisions):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.stack(v)
    T = V[np.array(faces)]
    # orient CCW seen from outside
    n = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
    flip = np.einsum("ij,ij->i", n, T.mean(axis=1)) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return T


def value_noise_heights(n_side: int, extent: float, h_max: float, rng: np.random.Generator,
                        octaves: int = 6, base_cells: int = 4):
    """Heights of an n_side x n_side vertex grid over [-extent/2, extent/2]^2.

    Octave o uses a lattice of base_cells * 2**o cells with U[0,1) values, a
    quintic fade and amplitude 0.5**o; the sum is min-max normalised to
    [0, h_max].  Returns (heights[n_side, n_side] f64 indexed [i_x, i_z],
    evaluate(x, z) for arbitrary points with the same normalisation).
    """
    lattices = [rng.random((base_cells * 2 ** o + 1, base_cells * 2 ** o + 1)) for o in range(octaves)]

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    def raw(u, w):  # u, w in [0, 1]
        acc = np.zeros(np.broadcast(u, w).shape)
        for o, lat in enumerate(lattices):
            cells = lat.shape[0] - 1
            x = np.clip(u, 0.0, 1.0) * cells
            z = np.clip(w, 0.0, 1.0) * cells
            i0 = np.minimum(np.floor(x).astype(np.int64), cells - 1)
            k0 = np.minimum(np.floor(z).astype(np.int64), cells - 1)
            fx, fz = fade(x - i0), fade(z - k0)
            a = lat[i0, k0] * (1 - fx) + lat[i0 + 1, k0] * fx
            b = lat[i0, k0 + 1] * (1 - fx) + lat[i0 + 1, k0 + 1] * fx
            acc += (0.5 ** o) * (a * (1 - fz) + b * fz)
        return acc

    g = np.linspace(0.0, 1.0, n_side)
    H = raw(g[:, None], g[None, :])
    lo, hi = H.min(), H.max()

    def evaluate(x, z):
        u = (np.asarray(x, dtype=np.float64) + extent / 2) / extent
        w = (np.asarray(z, dtype=np.float64) + extent / 2) / extent
        return (raw(u, w) - lo) / (hi - lo) * h_max

    return (H - lo) / (hi - lo) * h_max, evaluate


def heightfield_tris(heights: np.ndarray, extent: float) -> np.ndarray:
    """Grid heights [i_x, i_z] -> (2 (n-1)^2, 3, 3) triangles, CCW seen from +y."""
    n = heights.shape[0]
    xs = np.linspace(-extent / 2, extent / 2, n)
    X, Z = np.meshgrid(xs, xs, indexing="ij")
    P = np.stack([X, heights, Z], axis=-1)
    a = P[:-1, :-1].reshape(-1, 3)
    b = P[1:, :-1].reshape(-1, 3)
    c = P[:-1, 1:].reshape(-1, 3)
    d = P[1:, 1:].reshape(-1, 3)
    t1 = np.stack([a, c, b], axis=1)
    t2 = np.stack([b, c, d], axis=1)
    return np.stack([t1, t2], axis=1).reshape(-1, 3, 3)


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def config0(seed: int = 0) -> Workload:
    """128x128, 8 random Phong spheres + ground plane y=-5, one light, depth 3."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-4.0, 4.0, size=(8, 3))
    r = rng.uniform(0.3, 1.0, size=(8, 1))
    alb = rng.uniform(0.0, 1.0, size=(8, 3))
    mats = [material(tuple(alb[i]), k_a=0.1, k_d=1.0, k_s=0.5, shininess=32, k_r=0.3) for i in range(8)]
    mats.append(material((0.75, 0.75, 0.75), k_a=0.1, k_d=1.0, k_s=0.5, shininess=32, k_r=0.3))
    scene = make_scene(spheres=np.hstack([c, r]), sphere_mat=np.arange(8),
                       planes=[[0.0, 1.0, 0.0, -5.0]], plane_mat=[8],
                       materials=np.stack(mats), lights=[[5.0, 8.0, -5.0, 1.0, 1.0, 1.0]], name="c0_spheres")
    cam = Camera((0.0, 0.0, -10.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, 128, 128)
    return Workload(scene, cam, Params(spp=1, max_depth=3, jitter=0, seed=seed), "c0_spheres_128")


def config1(seed: int = 1, width: int = 1920, height: int = 1080, grid: int = 512) -> Workload:
    """1080p, 512x512-vertex value-noise terrain + 64 mirror spheres, 4 lights, depth 5."""
    rng = np.random.default_rng(seed)
    extent = 200.0
    heights, h_at = value_noise_heights(grid, extent, 20.0, rng)
    tris = heightfield_tris(heights, extent)
    ns = 64
    r = rng.uniform(1.0, 3.0, size=ns)
    xz = rng.uniform(-90.0, 90.0, size=(ns, 2))
    lift = rng.uniform(1.0, 10.0, size=ns)
    y = h_at(xz[:, 0], xz[:, 1]) + r + lift
    spheres = np.stack([xz[:, 0], y, xz[:, 1], r], axis=1)
    mats = np.stack([material((0.55, 0.5, 0.45), k_a=0.1, k_d=1.0, k_s=0.5, shininess=32, k_r=0.0),
                     mirror_material(0.9)])
    lights = [[sx * 60.0, 80.0, sz * 60.0, 0.25, 0.25, 0.25] for sx in (-1, 1) for sz in (-1, 1)]
    scene = make_scene(spheres=spheres, sphere_mat=np.ones(ns), tris=tris, tri_mat=np.zeros(len(tris)),
                       materials=mats, lights=lights, name="c1_terrain")
    cam = Camera((0.0, 60.0, -150.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, width, height)
    return Workload(scene, cam, Params(spp=1, max_depth=5, jitter=0, seed=seed), f"c1_terrain_{width}x{height}")


def config2(seed: int = 2, width: int = 1920, height: int = 1080, spp: int = 16, n_objects: int = 1000,
            subdivisions: int = 3) -> Workload:
    """1080p x 16 jittered spp, 1000 icospheres (1.28M tris), 50/30/20 Phong/mirror/glass, 8 lights, depth 8."""
    rng = np.random.default_rng(seed)
    unit = icosphere(subdivisions)
    centres = rng.uniform(-50.0, 50.0, size=(n_objects, 3))
    radii = rng.uniform(0.5, 2.0, size=n_objects)
    kind = rng.choice(3, size=n_objects, p=[0.5, 0.3, 0.2])
    alb = rng.uniform(0.0, 1.0, size=(n_objects, 3))
    tris = unit[None] * radii[:, None, None, None] + centres[:, None, None, :]
    tris = tris.reshape(-1, 3, 3)
    mats = []
    for i in range(n_objects):
        if kind[i] == 0:
            mats.append(material(tuple(alb[i]), k_a=0.1, k_d=1.0, k_s=0.5, shininess=32, k_r=0.0))
        elif kind[i] == 1:
            mats.append(mirror_material(0.9))
        else:
            mats.append(dielectric_material(1.5))
    tri_mat = np.repeat(np.arange(n_objects), len(unit))
    lights = [[sx * 70.0, sy * 70.0, sz * 70.0, 0.125, 0.125, 0.125]
              for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)]
    scene = make_scene(tris=tris, tri_mat=tri_mat, materials=np.stack(mats), lights=lights, name="c2_icospheres")
    cam = Camera((0.0, 0.0, -150.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, width, height)
    return Workload(scene, cam, Params(spp=spp, max_depth=8, jitter=1, seed=seed),
                    f"c2_icospheres_{width}x{height}x{spp}spp")


def config3_scene(b: int) -> Workload:
    """One scene of the 256-scene batch (seed 3000 + b)."""
    rng = np.random.default_rng(3000 + b)
    T = math.exp(rng.uniform(math.log(1e3), math.log(2e5)))
    side = int(round(math.exp(rng.uniform(math.log(64), math.log(512)))))
    depth = int(rng.integers(2, 7))
    if rng.random() < 0.5:
        n = max(1, int(round(T / 320)))
        s = (n / 8.0) ** (1.0 / 3.0)
        unit = icosphere(2)
        c = rng.uniform(-4.0 * s, 4.0 * s, size=(n, 3))
        r = rng.uniform(0.3, 1.0, size=n)
        alb = rng.uniform(0.0, 1.0, size=(n, 3))
        tris = (unit[None] * r[:, None, None, None] + c[:, None, None, :]).reshape(-1, 3, 3)
        mats = np.stack([material(tuple(alb[i]), k_r=0.3) for i in range(n)] +
                        [material((0.75, 0.75, 0.75), k_r=0.3)])
        scene = make_scene(tris=tris, tri_mat=np.repeat(np.arange(n), len(unit)),
                           planes=[[0.0, 1.0, 0.0, -5.0 * s]], plane_mat=[n], materials=mats,
                           lights=[[5.0 * s, 8.0 * s, -5.0 * s, 1.0, 1.0, 1.0]], name=f"c3_{b}_spheres")
        cam = Camera((0.0, 0.0, -10.0 * s), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, side, side)
    else:
        g = max(2, int(round(math.sqrt(T / 2.0))) + 1)
        heights, h_at = value_noise_heights(g, 200.0, 20.0, rng)
        tris = heightfield_tris(heights, 200.0)
        ns = 8
        r = rng.uniform(1.0, 3.0, size=ns)
        xz = rng.uniform(-90.0, 90.0, size=(ns, 2))
        y = h_at(xz[:, 0], xz[:, 1]) + r + rng.uniform(1.0, 10.0, size=ns)
        mats = np.stack([material((0.55, 0.5, 0.45), k_r=0.0), mirror_material(0.9)])
        lights = [[sx * 60.0, 80.0, sz * 60.0, 0.25, 0.25, 0.25] for sx in (-1, 1) for sz in (-1, 1)]
        scene = make_scene(spheres=np.stack([xz[:, 0], y, xz[:, 1], r], axis=1), sphere_mat=np.ones(ns),
                           tris=tris, tri_mat=np.zeros(len(tris)), materials=mats, lights=lights,
                           name=f"c3_{b}_terrain")
        cam = Camera((0.0, 60.0, -150.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, side, side)
    return Workload(scene, cam, Params(spp=1, max_depth=depth, jitter=0, seed=3000 + b), f"c3_{b}")


def config3(n: int = 256) -> List[Workload]:
    """The batch: n uneven scenes (log-uniform triangle counts and resolutions, depth 2..6)."""
    return [config3_scene(b) for b in range(n)]


# --------------------------------------------------------------------------
# Small scenes used by tests
# --------------------------------------------------------------------------

def one_sphere(center=(0.0, 0.0, 0.0), radius=1.0, plane_y: Optional[float] = None,
               light=(5.0, 8.0, -5.0), size=64, mat=None) -> Workload:
    mats = [material((0.8, 0.3, 0.2), k_r=0.0) if mat is None else mat, material((0.75, 0.75, 0.75), k_r=0.0)]
    planes, pmat = (None, None) if plane_y is None else ([[0.0, 1.0, 0.0, plane_y]], [1])
    scene = make_scene(spheres=[[*center, radius]], sphere_mat=[0], planes=planes, plane_mat=pmat,
                       materials=np.stack(mats), lights=[[*light, 1.0, 1.0, 1.0]], name="one_sphere")
    cam = Camera((0.0, 0.0, -10.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, size, size)
    return Workload(scene, cam, Params(spp=1, max_depth=0), "one_sphere")


def random_tiny(seed: int, n_spheres=4, n_tris=24, with_plane=True, size=24, depth=3) -> Workload:
    """Small mixed scene for BVH vs brute-force and full-image parity at every pixel."""
    rng = np.random.default_rng(10_000 + seed)
    sph = np.hstack([rng.uniform(-3, 3, size=(n_spheres, 3)), rng.uniform(0.3, 1.2, size=(n_spheres, 1))])
    cen = rng.uniform(-3, 3, size=(n_tris, 1, 3))
    tris = cen + rng.normal(0.0, 0.8, size=(n_tris, 3, 3))
    mats = np.stack([material(tuple(rng.uniform(0, 1, 3)), k_r=0.3),
                     mirror_material(0.9), dielectric_material(1.5),
                     material((0.75, 0.75, 0.75), k_r=0.0)])
    planes, pmat = ([[0.0, 1.0, 0.0, -4.0]], [3]) if with_plane else (None, None)
    scene = make_scene(spheres=sph, sphere_mat=rng.integers(0, 3, size=n_spheres),
                       tris=tris, tri_mat=rng.integers(0, 3, size=n_tris), planes=planes, plane_mat=pmat,
                       materials=mats, lights=[[4.0, 7.0, -6.0, 0.6, 0.6, 0.6], [-5.0, 6.0, -2.0, 0.4, 0.4, 0.4]],
                       name=f"tiny_{seed}")
    cam = Camera((0.0, 0.5, -11.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 55.0, size, size)
    return Workload(scene, cam, Params(spp=1, max_depth=depth, jitter=0, seed=seed), f"tiny_{seed}")


def pixel_subset(cam: Camera, n: int, seed: int) -> np.ndarray:
    """Seeded sample of distinct pixel indices (row-major, row 0 at the top)."""
    rng = np.random.default_rng(seed)
    n = min(n, cam.n_pixels)
    return np.sort(rng.choice(cam.n_pixels, size=n, replace=False)).astype(np.int64)


def with_disk_lights(w: Workload, radius: float) -> Workload:
    """The same workload with each point light replaced by a disk of the given radius centred on it and
    facing the scene origin (area lights sampled once per pass)."""
    import copy
    w = copy.deepcopy(w)
    L = w.scene.lights.copy()
    for i in range(len(L)):
        n = -L[i, :3].astype(np.float64)
        n /= max(np.linalg.norm(n), 1e-30)
        a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        u = np.cross(n, a)
        u /= np.linalg.norm(u)
        v = np.cross(n, u)
        L[i, 6] = DISK
        L[i, 7:10] = radius * u
        L[i, 10:13] = radius * v
    w.scene.lights = L.astype(np.float32)
    w.name = w.name + f"_disk{radius:g}"
    return w


def mlp_init_weights(seed: int):
    """He-uniform FP32 initial weights of the radiance-cache network from a seeded RNG:
    [W1 .. W5] (64 x 64, row-major out x in), W6 (3 x 64).  The fan-in of W1 counts the
    42 real input features; its columns for the zero padding are zero."""
    rng = np.random.default_rng(seed)
    ws = []
    for l in range(5):
        fan = 42 if l == 0 else 64
        b = math.sqrt(6.0 / fan)
        w = rng.uniform(-b, b, size=(64, 64))
        if l == 0:
            w[:, 42:] = 0.0
        ws.append(w.astype(np.float32))
    b = math.sqrt(6.0 / 64)
    ws.append(rng.uniform(-b, b, size=(3, 64)).astype(np.float32))
    return ws


def config4(seed: int = 2, **kw) -> Workload:
    """The learned form's workload: the c2 scene, camera and samples (plain reference at depth 8)."""
    w = config2(seed, **kw)
    w.name = w.name.replace("c2_", "c4_cache_")
    return w


def config_gi(seed: int = 2, max_depth: int = 6, **kw) -> Workload:
    """Diffuse global illumination at path depth 6 (the depth of the paper's global-illumination image): the
    c2 scene, camera, lights and samples inside a closed room of six Lambert walls (x = +-80, y = +-80,
    z = -160 and 80; grey, one red and one green side wall), so that no path escapes before its last bounce."""
    w = config2(seed, **kw)
    sc = w.scene
    n_mat = len(sc.materials)
    walls = np.stack([material((0.75, 0.25, 0.25), k_a=0.05, k_d=1.0, k_s=0.0),
                      material((0.25, 0.75, 0.25), k_a=0.05, k_d=1.0, k_s=0.0),
                      material((0.75, 0.75, 0.75), k_a=0.05, k_d=1.0, k_s=0.0)])
    planes = [[1.0, 0.0, 0.0, -80.0], [1.0, 0.0, 0.0, 80.0], [0.0, 1.0, 0.0, -80.0], [0.0, 1.0, 0.0, 80.0],
              [0.0, 0.0, 1.0, -160.0], [0.0, 0.0, 1.0, 80.0]]
    plane_mat = [n_mat, n_mat + 1, n_mat + 2, n_mat + 2, n_mat + 2, n_mat + 2]
    scene = make_scene(tris=sc.tris, tri_mat=sc.tri_mat, planes=planes, plane_mat=plane_mat,
                       materials=np.concatenate([sc.materials, walls]), lights=sc.lights, name="gi_room_icospheres")
    p = w.params
    p.gi, p.max_depth = 1, max_depth
    cam = w.camera
    return Workload(scene, cam, p, f"gi_room_icospheres_{cam.width}x{cam.height}x{p.spp}spp_depth{max_depth}")


WORKLOADS = {"c0": config0, "c1": config1, "c2": config2, "c4": config4, "gi": config_gi}
