"""FP64 CPU oracle for the ray tracer.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library
(``paper_1504_03151_amd``) never imports it and shares no code with it; the
only common inputs are the scenes from ``paper_1504_03151_amd.scenes``, which
hold none of the tracer's arithmetic.

``oracle.c`` is the brute-force Whitted tracer (Algorithm 1 plus the recursive
extension of Section III/IV.A, sphere roots by Eq. 11-12); ``mlp.py`` is the
radiance-cache network's forward/backward/Adam in FP64 with BF16 rounding
emulation.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

BUILD_CMD = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-o", _LIB, _SRC,
             "-lm", "-lpthread"]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (seconds)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = list(BUILD_CMD)
        cmd[cmd.index(_LIB)] = tmp
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [("n_spheres", C.c_int64), ("spheres", C.c_void_p), ("sphere_mat", C.c_void_p),
                ("n_tris", C.c_int64), ("tris", C.c_void_p), ("tri_mat", C.c_void_p),
                ("n_planes", C.c_int64), ("planes", C.c_void_p), ("plane_mat", C.c_void_p),
                ("n_materials", C.c_int32), ("materials", C.c_void_p),
                ("n_lights", C.c_int32), ("lights", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("look_at", C.c_double * 3), ("up", C.c_double * 3),
                ("vfov_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("spp", C.c_int32), ("max_depth", C.c_int32), ("jitter", C.c_int32), ("gi", C.c_int32),
                ("seed", C.c_uint64), ("frame", C.c_uint32), ("pad1", C.c_uint32),
                ("bg", C.c_double * 3), ("eps", C.c_double)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = C.CDLL(build())
            L.or_render.restype = C.c_int
            L.or_render.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Params), C.c_void_p,
                                    C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]
            L.or_closest.restype = C.c_int
            L.or_closest.argtypes = [C.POINTER(_Scene), C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]
            L.or_occluded.restype = C.c_int
            L.or_occluded.argtypes = [C.POINTER(_Scene), C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                      C.c_void_p]
            L.or_camera_ray.restype = None
            L.or_camera_ray.argtypes = [C.POINTER(_Camera), C.POINTER(_Params), C.c_int64, C.c_int32,
                                        C.c_void_p, C.c_void_p]
            L.or_ray_tree.restype = C.c_int64
            L.or_ray_tree.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Params), C.c_int64,
                                      C.c_int32, C.c_void_p, C.c_int64, C.c_void_p]
            L.or_render_cache.restype = C.c_int64
            L.or_render_cache.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Params), C.c_void_p,
                                          C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_int64]
            L.or_radiance.restype = C.c_int
            L.or_radiance.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), C.c_void_p, C.c_int64, C.c_int32,
                                      C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
            L.or_light_point.restype = None
            L.or_light_point.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_int32, C.c_int32, C.c_void_p]
            L.or_pcg.restype = C.c_uint32
            L.or_pcg.argtypes = [C.c_uint32]
            L.or_jitter.restype = C.c_double
            L.or_jitter.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
            L.or_path_rand.restype = C.c_double
            L.or_path_rand.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
            _lib = L
    return _lib


class OScene:
    """Keeps the scene arrays alive while the C structure points at them."""

    def __init__(self, scene):
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a.ctypes.data if a.size else None

        s = _Scene()
        s.n_spheres = len(scene.spheres)
        s.spheres = arr(scene.spheres, np.float32)
        s.sphere_mat = arr(scene.sphere_mat, np.int32)
        s.n_tris = len(scene.tris)
        s.tris = arr(scene.tris, np.float32)
        s.tri_mat = arr(scene.tri_mat, np.int32)
        s.n_planes = len(scene.planes)
        s.planes = arr(scene.planes, np.float32)
        s.plane_mat = arr(scene.plane_mat, np.int32)
        s.n_materials = len(scene.materials)
        s.materials = arr(scene.materials, np.float32)
        s.n_lights = len(scene.lights)
        s.lights = arr(scene.lights, np.float32)
        self.c = s


def _camera(cam) -> _Camera:
    c = _Camera()
    c.eye[:] = [float(x) for x in cam.eye]
    c.look_at[:] = [float(x) for x in cam.look_at]
    c.up[:] = [float(x) for x in cam.up]
    c.vfov_deg = float(cam.vfov_deg)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _params(p) -> _Params:
    q = _Params()
    q.spp, q.max_depth, q.jitter = int(p.spp), int(p.max_depth), int(p.jitter)
    q.gi = int(getattr(p, "gi", 0))
    q.seed, q.frame = int(p.seed) & (2 ** 64 - 1), int(p.frame) & (2 ** 32 - 1)
    q.bg[:] = [float(x) for x in p.bg]
    q.eps = float(p.eps)
    return q


def render(scene, camera, params, pixels=None, nthreads: int = 0):
    """Brute-force render of the given pixels (default: all).

    Returns dict(rgb [n,3] f64, ids [n,spp] i64, margin [n] f64, counts [n,D+1,2] i32, pixels [n] i64,
    rgb_s [n,spp,3] f64 per-sample radiance, margin_s [n,spp] per-sample margin).
    """
    L = lib()
    if pixels is None:
        pixels = np.arange(camera.width * camera.height, dtype=np.int64)
    pixels = np.ascontiguousarray(pixels, dtype=np.int64)
    n = len(pixels)
    D = int(params.max_depth)
    rgb = np.zeros((n, 3), np.float64)
    ids = np.zeros((n, params.spp), np.int64)
    margin = np.zeros((n,), np.float64)
    counts = np.zeros((n, D + 1, 2), np.int32)
    rgb_s = np.zeros((n, params.spp, 3), np.float64)
    margin_s = np.zeros((n, params.spp), np.float64)
    sc, cam, p = OScene(scene), _camera(camera), _params(params)
    rc = L.or_render(C.byref(sc.c), C.byref(cam), C.byref(p), pixels.ctypes.data, n, nthreads,
                     rgb.ctypes.data, ids.ctypes.data, margin.ctypes.data, counts.ctypes.data,
                     rgb_s.ctypes.data, margin_s.ctypes.data)
    if rc != 0:
        raise ValueError(f"or_render failed ({rc})")
    return dict(rgb=rgb, ids=ids, margin=margin, counts=counts, pixels=pixels, rgb_s=rgb_s, margin_s=margin_s)


def _rays9(o, d, tmax=None, so=0.0, sd=0.0):
    o = np.asarray(o, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64).reshape(-1, 3)
    n = len(o)
    R = np.zeros((n, 9), np.float64)
    R[:, 0:3] = o
    R[:, 3:6] = d
    R[:, 6] = 0.0 if tmax is None else np.broadcast_to(np.asarray(tmax, np.float64), (n,))
    R[:, 7] = so
    R[:, 8] = sd
    return R


def closest(scene, o, d, tmax=None, so=0.0, sd=0.0, nthreads: int = 0, uv: bool = False):
    """Brute-force closest hit. tmax None/<=0 = infinite. Returns (t, id, margin), and with uv=True
    also the hit's surface coordinates [n, 2] (triangle barycentrics of v1 and v2; sphere longitude
    and polar angle of the outward normal over 2 pi and pi; 0 for planes and misses)."""
    L = lib()
    R = _rays9(o, d, tmax, so, sd)
    n = len(R)
    t = np.zeros(n, np.float64)
    ids = np.zeros(n, np.int64)
    m = np.zeros(n, np.float64)
    huv = np.zeros((n, 2), np.float64) if uv else None
    sc = OScene(scene)
    L.or_closest(C.byref(sc.c), R.ctypes.data, n, nthreads, t.ctypes.data, ids.ctypes.data, m.ctypes.data,
                 huv.ctypes.data if uv else None)
    return (t, ids, m, huv) if uv else (t, ids, m)


def occluded(scene, o, d, tmax, so=0.0, sd=0.0, nthreads: int = 0):
    """Brute-force any-hit on (0, tmax). Returns (occluded bool, margin)."""
    L = lib()
    R = _rays9(o, d, tmax, so, sd)
    n = len(R)
    occ = np.zeros(n, np.uint8)
    m = np.zeros(n, np.float64)
    sc = OScene(scene)
    L.or_occluded(C.byref(sc.c), R.ctypes.data, n, nthreads, occ.ctypes.data, m.ctypes.data)
    return occ.astype(bool), m


def camera_rays(camera, params, pixels, sample: int = 0):
    """FP64 primary rays for the given pixels and sample index: (o [n,3], d [n,3])."""
    L = lib()
    pixels = np.asarray(pixels, np.int64).reshape(-1)
    o = np.zeros((len(pixels), 3), np.float64)
    d = np.zeros((len(pixels), 3), np.float64)
    cam, p = _camera(camera), _params(params)
    buf_o = (C.c_double * 3)()
    buf_d = (C.c_double * 3)()
    for i, px in enumerate(pixels):
        L.or_camera_ray(C.byref(cam), C.byref(p), int(px), int(sample), buf_o, buf_d)
        o[i] = list(buf_o)
        d[i] = list(buf_d)
    return o, d


RAY_KIND = {0: "camera", 1: "reflected", 2: "refracted", 3: "shadow"}


def ray_tree(scene, camera, params, pixel: int, sample: int = 0, cap: int = 4096):
    """Every ray the oracle traces for one pixel sample, in recursion order.

    Returns (records [n, 12] f64, rgb [3]); record columns: kind (0 camera,
    1 reflected, 2 refracted, 3 shadow), depth, o[3], d[3], tmax, t (closest
    hit; for shadow rays 1.0 if blocked else 0.0), id, margin.
    """
    L = lib()
    rec = np.zeros((cap, 12), np.float64)
    rgb = np.zeros(3, np.float64)
    sc, cam, p = OScene(scene), _camera(camera), _params(params)
    n = L.or_ray_tree(C.byref(sc.c), C.byref(cam), C.byref(p), int(pixel), int(sample), rec.ctypes.data, cap,
                      rgb.ctypes.data)
    if n < 0:
        raise ValueError(f"or_ray_tree failed ({n})")
    if n > cap:
        raise ValueError(f"ray tree has {n} rays > cap {cap}")
    return rec[:n].copy(), rgb


def pcg(v: int) -> int:
    return int(lib().or_pcg(v & 0xFFFFFFFF))


def jitter(seed: int, frame: int, pixel: int, s: int, dim: int) -> float:
    return float(lib().or_jitter(seed & (2 ** 64 - 1), frame, pixel, s, dim))


def path_rand(seed: int, frame: int, pixel: int, s: int, depth: int, k: int) -> float:
    """Random number k of the bounce at `depth` of sample s of a pixel (global illumination paths)."""
    return float(lib().or_path_rand(seed & (2 ** 64 - 1), frame, pixel, s, depth, k))


ROBUST = 1e-4


def render_cache(scene, camera, params, cache_depth: int, pixels=None, nthreads: int = 0, cap: int = 1 << 22):
    """Learned-form render without the cache terms: dict(rgb [n,3], margin [n], records [m,13]).

    Each record (list index, x[3], N_f[3], V[3], w[3]) is a hit at cache_depth whose
    radiance the cache supplies: pixel += w * max(cache(x, N_f, V), 0) / spp.
    """
    L = lib()
    if pixels is None:
        pixels = np.arange(camera.width * camera.height, dtype=np.int64)
    pixels = np.ascontiguousarray(pixels, dtype=np.int64)
    n = len(pixels)
    rgb = np.zeros((n, 3), np.float64)
    margin = np.zeros((n,), np.float64)
    rec = np.zeros((cap, 13), np.float64)
    sc, cam, p = OScene(scene), _camera(camera), _params(params)
    m = L.or_render_cache(C.byref(sc.c), C.byref(cam), C.byref(p), pixels.ctypes.data, n, int(cache_depth), nthreads,
                          rgb.ctypes.data, margin.ctypes.data, rec.ctypes.data, cap)
    if m < 0 or m > cap:
        raise ValueError(f"or_render_cache failed ({m})")
    return dict(rgb=rgb, margin=margin, records=rec[:m].copy(), pixels=pixels)


def radiance(scene, params, o, d, start_depth: int, so=0.0, sd=0.0, nthreads: int = 0, sample: int = 0,
             pixels=None):
    """Radiance of rays starting at recursion depth start_depth: (L [n,3], margin [n]); area lights take their
    points of pass `sample`; with global illumination ray i's path is keyed by pixels[i] (default: i)."""
    Lb = lib()
    R = _rays9(o, d, None, so, sd)
    n = len(R)
    out = np.zeros((n, 3), np.float64)
    m = np.zeros(n, np.float64)
    sc, p = OScene(scene), _params(params)
    px = None if pixels is None else np.ascontiguousarray(pixels, np.int64).reshape(n)
    rc = Lb.or_radiance(C.byref(sc.c), C.byref(p), R.ctypes.data, n, int(start_depth), int(sample), nthreads,
                        out.ctypes.data, m.ctypes.data, None if px is None else px.ctypes.data)
    if rc != 0:
        raise ValueError(f"or_radiance failed ({rc})")
    return out, m


def light_point(light, seed: int, frame: int, sample: int, index: int):
    """Sample point of one light record (13 floats) for a pass (frame, sample) and light index."""
    L = np.ascontiguousarray(light, np.float32).reshape(13)
    out = np.zeros(3, np.float64)
    lib().or_light_point(L.ctypes.data, int(seed) & (2 ** 64 - 1), int(frame), int(sample), int(index),
                         out.ctypes.data)
    return out
