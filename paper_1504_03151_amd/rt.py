"""Thin Python binding of libmirt.so (include/mirt.h).

Argument marshalling only: every step of the tracer runs in the HIP library.
torch provides device memory and the HIP stream.  If the library is missing
this module raises at import-time use (``lib()``); there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MIRT_LIB") or os.path.join(_HERE, "libmirt.so")   # MIRT_LIB: another build of it
_lock = threading.Lock()
_lib = None

RT_OK = 0
RT_ERR = {-1: "INVALID_ARG", -2: "UNSUPPORTED", -3: "HIP", -4: "BVH_DEPTH", -5: "CAPACITY",
          -6: "DEVICE_STATUS", -7: "NOT_UPLOADED"}
FLAG_SYNC, FLAG_COUNT_WORK, FLAG_NO_GRAPH, FLAG_TIME_KERNELS, FLAG_PER_SAMPLE = 1, 2, 4, 8, 16
FLAG_ACCUMULATE = 32
FLAG_GI = 64            # diffuse global illumination by path tracing (set from Params.gi)
FLAG_TIME_SHADOW = 128  # HIP events around the shadow launches only
STATS_MAX_DEPTH = 16


class RTError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn} failed: RT_ERR_{RT_ERR.get(status, status)} ({status}): {msg}")
        self.status = status


class Material(C.Structure):
    _fields_ = [("albedo", C.c_float * 3), ("k_a", C.c_float), ("k_d", C.c_float), ("k_s", C.c_float),
                ("shininess", C.c_float), ("k_r", C.c_float), ("ior", C.c_float), ("type", C.c_int32)]


class Light(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("intensity", C.c_float * 3), ("shape", C.c_int32), ("u", C.c_float * 3),
                ("v", C.c_float * 3)]


class SceneDesc(C.Structure):
    _fields_ = [("spheres", C.c_void_p), ("n_spheres", C.c_int64), ("sphere_mat", C.c_void_p),
                ("tris", C.c_void_p), ("n_tris", C.c_int64), ("tri_mat", C.c_void_p),
                ("planes", C.c_void_p), ("n_planes", C.c_int64), ("plane_mat", C.c_void_p),
                ("materials", C.c_void_p), ("n_materials", C.c_int32),
                ("lights", C.c_void_p), ("n_lights", C.c_int32)]


class BuildOpts(C.Structure):
    _fields_ = [("leaf_max", C.c_int32), ("sah_bins", C.c_int32), ("max_depth", C.c_int32),
                ("node_layout", C.c_int32)]


class CameraC(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class ParamsC(C.Structure):
    _fields_ = [("spp", C.c_int32), ("max_depth", C.c_int32), ("jitter", C.c_int32), ("frame", C.c_uint32),
                ("seed", C.c_uint64), ("bg", C.c_float * 3), ("eps", C.c_float),
                ("samples_per_pass", C.c_int32), ("flags", C.c_int32), ("queue_factor", C.c_float),
                ("queue_chunk", C.c_int32), ("tile", C.c_int32), ("accum_frames", C.c_uint32),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("stats", C.c_void_p), ("stream", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_uint32), ("passes", C.c_uint32),
                ("rays", C.c_uint64 * STATS_MAX_DEPTH), ("shadow", C.c_uint64 * STATS_MAX_DEPTH),
                ("node_visits", C.c_uint64), ("tri_tests", C.c_uint64), ("sphere_tests", C.c_uint64),
                ("shadow_node_visits", C.c_uint64), ("shadow_tri_tests", C.c_uint64),
                ("shadow_sphere_tests", C.c_uint64), ("cache_queries", C.c_uint64), ("target_rays", C.c_uint64),
                ("target_shadow", C.c_uint64)]


class SceneInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("depth", C.c_int32), ("stack_size", C.c_int32),
                ("n_leaves", C.c_int64), ("n_bvh_prims", C.c_int64), ("sah_cost", C.c_double),
                ("build_seconds", C.c_double), ("bounds_lo", C.c_float * 3), ("bounds_hi", C.c_float * 3),
                ("node_layout", C.c_int32)]


class CacheC(C.Structure):
    _fields_ = [("mode", C.c_int32), ("depth", C.c_int32), ("full_depth", C.c_int32), ("train_samples", C.c_int32),
                ("train_steps", C.c_int32), ("lr", C.c_float), ("b1", C.c_float), ("b2", C.c_float),
                ("eps", C.c_float), ("bounds_lo", C.c_float * 3), ("bounds_hi", C.c_float * 3),
                ("state", C.c_void_p)]


class CacheLayout(C.Structure):
    _fields_ = [(k, C.c_size_t) for k in ("w_master", "w_bf16", "m", "v", "grad", "counters", "train_rays",
                                           "train_feats", "train_targets", "train_pix", "total")] + [("capacity", C.c_int32)]


CACHE_INFER, CACHE_TRAIN = 1, 2
CACHE_HEALTH_LOSS, CACHE_HEALTH_WEIGHTS, CACHE_HEALTH_BF16 = 1, 2, 4
STATUS_RAY_OVERFLOW, STATUS_SHADOW_OVERFLOW, STATUS_CACHE_RECORDS, STATUS_CACHE_FALLBACK = 1, 2, 4, 8
LAYOUT_DFS, LAYOUT_BFS, LAYOUT_TREELET, LAYOUT_BVH4, LAYOUT_BVH4Q = 0, 1, 2, 3, 4
NODE_BYTES = {0: 64, 1: 64, 2: 64, 3: 128, 4: 64}   # bytes fetched per node visit, by layout
TILE_8X8, TILE_16X4, TILE_32X2, TILE_4X16 = 0, 1, 2, 3
TILE_SHAPES = {TILE_8X8: (8, 8), TILE_16X4: (16, 4), TILE_32X2: (32, 2), TILE_4X16: (4, 16)}

# every symbol include/mirt.h declares: name -> (restype, argtypes)
_P = C.c_void_p
SIGNATURES = {
    "rt_build_scene": (C.c_int32, [C.POINTER(SceneDesc), C.POINTER(BuildOpts), C.POINTER(C.c_void_p)]),
    "rt_destroy_scene": (None, [_P]),
    "rt_scene_get_info": (C.c_int32, [_P, C.POINTER(SceneInfo)]),
    "rt_scene_set_layout": (C.c_int32, [_P, C.c_int32]),
    "rt_scene_device_bytes": (C.c_size_t, [_P]),
    "rt_scene_upload": (C.c_int32, [_P, _P, C.c_size_t, _P]),
    "rt_scene_refit_workspace_bytes": (C.c_size_t, [_P]),
    "rt_scene_refit": (C.c_int32, [_P, _P, _P, _P, C.c_size_t, C.c_int32, _P]),
    "rt_scene_refit_noalloc_max_bytes": (C.c_size_t, []),
    "rt_scene_refit_noalloc": (C.c_int32, [_P, _P, _P, C.c_int32, _P]),
    "rt_render_workspace_bytes": (C.c_size_t, [_P, C.POINTER(CameraC), C.POINTER(ParamsC)]),
    "rt_render": (C.c_int32, [_P, C.POINTER(CameraC), C.POINTER(ParamsC), _P, _P]),
    "rt_render_batch_workspace_bytes": (C.c_size_t, [_P, _P, _P, C.c_int32]),
    "rt_render_batch": (C.c_int32, [_P, _P, _P, C.c_int32, _P, _P]),
    "rt_intersect": (C.c_int32, [_P, _P, C.c_int64, _P, _P, _P, _P, _P]),
    "rt_occluded": (C.c_int32, [_P, _P, C.c_int64, _P, _P, _P]),
    "rt_host_trace": (C.c_int32, [_P, _P, C.c_int64, C.c_int32, _P, _P, _P, C.c_int32]),
    "rt_kernel_times": (C.c_int32, [_P, _P, C.c_int32]),
    "rt_mlp_num_params": (C.c_int32, []),
    "rt_mlp_forward": (C.c_int32, [_P, _P, C.c_int64, _P, _P]),
    "rt_mlp_grad": (C.c_int32, [_P, _P, _P, C.c_int64, C.c_int64, _P, _P, _P]),
    "rt_mlp_adam": (C.c_int32, [_P, _P, _P, _P, _P, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, _P]),
    "rt_cache_state_layout": (C.c_int32, [C.c_int32, C.POINTER(CacheLayout)]),
    "rt_cache_state_bytes": (C.c_size_t, [C.c_int32]),
    "rt_cache_init": (C.c_int32, [_P, C.c_int32, _P, _P]),
    "rt_render_cached_workspace_bytes": (C.c_size_t, [_P, C.POINTER(CameraC), C.POINTER(ParamsC),
                                                      C.POINTER(CacheC)]),
    "rt_render_cached": (C.c_int32, [_P, C.POINTER(CameraC), C.POINTER(ParamsC), C.POINTER(CacheC), _P, _P]),
    "rt_last_error": (C.c_char_p, []),
    "rt_version": (C.c_char_p, []),
}


def lib():
    """Load libmirt.so; raises if it has not been built (no fallback)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  f"`python -m paper_1504_03151_amd.csrc.build` (needs ROCm hipcc)")
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def _check(status: int, fn: str):
    if status != RT_OK:
        raise RTError(status, fn, lib().rt_last_error().decode(errors="replace"))


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream_ptr(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream) or None


class Scene:
    """A built scene (host BVH + packed blob); upload() copies it to the GPU."""

    def __init__(self, scene, leaf_max: int = 0, sah_bins: int = 0, max_depth: int = 0, node_layout: int = 0):
        L = lib()
        self.src = scene
        keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a.ctypes.data if a.size else None

        mats = (Material * max(1, len(scene.materials)))()
        for i, m in enumerate(np.asarray(scene.materials, np.float32)):
            mats[i].albedo[:] = [float(x) for x in m[0:3]]
            mats[i].k_a, mats[i].k_d, mats[i].k_s, mats[i].shininess, mats[i].k_r, mats[i].ior = [
                float(x) for x in m[3:9]]
            mats[i].type = int(m[9])
        lights = (Light * max(1, len(scene.lights)))()
        for i, l in enumerate(np.asarray(scene.lights, np.float32)):
            lights[i].pos[:] = [float(x) for x in l[0:3]]
            lights[i].intensity[:] = [float(x) for x in l[3:6]]
            if len(l) > 6:
                lights[i].shape = int(l[6])
                lights[i].u[:] = [float(x) for x in l[7:10]]
                lights[i].v[:] = [float(x) for x in l[10:13]]
        d = SceneDesc()
        d.spheres, d.n_spheres, d.sphere_mat = arr(scene.spheres, np.float32), len(scene.spheres), arr(
            scene.sphere_mat, np.int32)
        d.tris, d.n_tris, d.tri_mat = arr(scene.tris, np.float32), len(scene.tris), arr(scene.tri_mat, np.int32)
        d.planes, d.n_planes, d.plane_mat = arr(scene.planes, np.float32), len(scene.planes), arr(
            scene.plane_mat, np.int32)
        d.materials, d.n_materials = C.cast(mats, C.c_void_p), len(scene.materials)
        d.lights, d.n_lights = C.cast(lights, C.c_void_p), len(scene.lights)
        opts = BuildOpts(leaf_max, sah_bins, max_depth, node_layout)
        h = C.c_void_p()
        _check(L.rt_build_scene(C.byref(d), C.byref(opts), C.byref(h)), "rt_build_scene")
        self.handle = h
        self.blob = None
        self._read_info()

    def _read_info(self):
        info = SceneInfo()
        _check(lib().rt_scene_get_info(self.handle, C.byref(info)), "rt_scene_get_info")
        self.info = {k: (list(getattr(info, k)) if k.startswith("bounds") else getattr(info, k))
                     for k, _ in SceneInfo._fields_}

    def set_layout(self, node_layout: int):
        """Reorder the BVH nodes (LAYOUT_*); the device copy is dropped, upload() again before rendering."""
        _check(lib().rt_scene_set_layout(self.handle, int(node_layout)), "rt_scene_set_layout")
        self.blob = None
        self._read_info()
        return self

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().rt_destroy_scene(self.handle)
                self.handle = None
        except Exception:
            pass

    @property
    def device_bytes(self) -> int:
        return int(lib().rt_scene_device_bytes(self.handle))

    def upload(self, device="cuda", stream=None):
        import torch
        n = self.device_bytes
        self.blob = torch.empty(n + 256, dtype=torch.uint8, device=device)
        base = (self.blob.data_ptr() + 255) // 256 * 256
        _check(lib().rt_scene_upload(self.handle, base, n, _stream_ptr(stream)), "rt_scene_upload")
        return self

    @property
    def device_base(self) -> int:
        """Device address of the uploaded blob (256-byte aligned inside self.blob)."""
        return (self.blob.data_ptr() + 255) // 256 * 256

    def device_blob(self):
        """The uploaded blob as a uint8 tensor view (rt_scene_device_bytes bytes)."""
        off = self.device_base - self.blob.data_ptr()
        return self.blob[off:off + self.device_bytes]

    def refit(self, spheres=None, tris=None, sync: bool = False, stream=None, noalloc: bool = False):
        """Refit the uploaded BVH on the GPU to new positions: spheres float32 [ns,4], tris float32 [nt,3,3]
        (contiguous CUDA tensors in the build order).  The tree is kept; only the device copy changes.
        noalloc=True: rt_scene_refit_noalloc (scratch in the library's static device buffer, no workspace)."""
        import torch
        if self.blob is None:
            raise RTError(-7, "rt_scene_refit", "scene not uploaded")
        ns, nt = len(self.src.spheres), len(self.src.tris)
        for t, n, what in ((spheres, 4 * ns, "spheres"), (tris, 9 * nt, "tris")):
            if n and (t is None or t.numel() != n):
                raise ValueError(f"refit: {what} must hold {n} floats")
            if t is not None:
                assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        flags = FLAG_SYNC if sync else 0
        if noalloc:
            _check(lib().rt_scene_refit_noalloc(self.handle, _ptr(spheres), _ptr(tris), flags, _stream_ptr(stream)),
                   "rt_scene_refit_noalloc")
            return self
        need = int(lib().rt_scene_refit_workspace_bytes(self.handle))
        ws = getattr(self, "_refit_ws", None)
        if ws is None or ws.numel() < need + 256:
            ws = self._refit_ws = torch.empty(need + 256, dtype=torch.uint8, device=self.blob.device)
        base = (ws.data_ptr() + 255) // 256 * 256
        _check(lib().rt_scene_refit(self.handle, _ptr(spheres), _ptr(tris), base, need, flags, _stream_ptr(stream)),
               "rt_scene_refit")
        return self

    def host_trace(self, rays: np.ndarray, any_hit: bool = False, nthreads: int = 0, with_work: bool = False):
        """Host FP32 traversal of the packed BVH. rays [n,8] f32 -> (t, id[, work [n,3]])."""
        rays = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
        n = len(rays)
        t = np.zeros(n, np.float32)
        ids = np.zeros(n, np.int32)
        work = np.zeros((n, 3), np.uint32) if with_work else None
        _check(lib().rt_host_trace(self.handle, rays.ctypes.data, n, int(any_hit), t.ctypes.data, ids.ctypes.data,
                                   None if work is None else work.ctypes.data, nthreads), "rt_host_trace")
        return (t, ids, work) if with_work else (t, ids)


def camera_c(cam) -> CameraC:
    c = CameraC()
    c.eye[:] = [float(x) for x in cam.eye]
    c.look_at[:] = [float(x) for x in cam.look_at]
    c.up[:] = [float(x) for x in cam.up]
    c.vfov_deg = float(cam.vfov_deg)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def params_c(p, flags=0, samples_per_pass=0, queue_factor=0.0, queue_chunk=0, tile=0) -> ParamsC:
    q = ParamsC()
    q.spp, q.max_depth, q.jitter, q.frame = int(p.spp), int(p.max_depth), int(p.jitter), int(p.frame)
    q.seed = int(p.seed) & (2 ** 64 - 1)
    q.bg[:] = [float(x) for x in p.bg]
    q.eps = float(p.eps)
    q.samples_per_pass = int(samples_per_pass)
    q.flags = int(flags) | (FLAG_GI if getattr(p, "gi", 0) else 0)
    q.queue_factor = float(queue_factor)
    q.queue_chunk = int(queue_chunk)
    q.tile = int(tile)
    return q


def stats_dict(buf) -> dict:
    """Decode an rt_stats device buffer (torch uint8 tensor)."""
    raw = buf.detach().cpu().numpy().tobytes()
    s = Stats.from_buffer_copy(raw[:C.sizeof(Stats)])
    return {"status": s.status, "passes": s.passes, "rays": list(s.rays), "shadow": list(s.shadow),
            "node_visits": s.node_visits, "tri_tests": s.tri_tests, "sphere_tests": s.sphere_tests,
            "shadow_node_visits": s.shadow_node_visits, "shadow_tri_tests": s.shadow_tri_tests,
            "shadow_sphere_tests": s.shadow_sphere_tests, "cache_queries": s.cache_queries,
            "target_rays": s.target_rays, "target_shadow": s.target_shadow}


class Renderer:
    """Owns the device workspace, outputs and stats for repeated frames of one scene/camera."""

    def __init__(self, scene: Scene, camera, params, device="cuda", with_ids=True, samples_per_pass=0,
                 queue_factor=0.0, graph=True, per_sample=False, queue_chunk=0, tile=0):
        import torch
        if scene.blob is None:
            scene.upload(device)
        self.scene, self.camera, self.params = scene, camera, params
        self.device = device
        self.samples_per_pass, self.queue_factor, self.graph = samples_per_pass, queue_factor, graph
        self.base_flags = FLAG_PER_SAMPLE if per_sample else 0
        self.queue_chunk, self.tile = queue_chunk, tile
        self.cam_c = camera_c(camera)
        self._alloc(with_ids)

    def _alloc(self, with_ids):
        import torch
        p = params_c(self.params, self.base_flags, self.samples_per_pass, self.queue_factor, tile=self.tile)
        n = lib().rt_render_workspace_bytes(self.scene.handle, C.byref(self.cam_c), C.byref(p))
        if n == 0:
            raise RTError(-1, "rt_render_workspace_bytes", lib().rt_last_error().decode())
        self.ws_bytes = int(n)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        H, W = self.camera.height, self.camera.width
        shape = (H, W, self.params.spp, 3) if self.base_flags & FLAG_PER_SAMPLE else (H, W, 3)
        self.rgb = torch.empty(shape, dtype=torch.float32, device=self.device)
        self.ids = torch.empty((H, W, self.params.spp), dtype=torch.int32, device=self.device) if with_ids else None
        self.stats = torch.zeros(C.sizeof(Stats) + 64, dtype=torch.uint8, device=self.device)

    def render(self, flags=0, stream=None, reset_stats=True, accum_frames=None):
        """One frame.  accum_frames=n: progressive mode, add this frame to the n frames already accumulated in
        this renderer's workspace (0 starts afresh) and return the running average."""
        if reset_stats:
            self.stats.zero_()
        if not self.graph:
            flags |= FLAG_NO_GRAPH
        if accum_frames is not None:
            flags |= FLAG_ACCUMULATE
        p = params_c(self.params, flags | self.base_flags, self.samples_per_pass, self.queue_factor,
                     self.queue_chunk, self.tile)
        p.accum_frames = int(accum_frames or 0)
        p.workspace, p.workspace_bytes = self.ws.data_ptr(), self.ws_bytes
        p.stats = self.stats.data_ptr()
        p.stream = _stream_ptr(stream)
        _check(lib().rt_render(self.scene.handle,
                               C.byref(self.cam_c), C.byref(p), self.rgb.data_ptr(), _ptr(self.ids)), "rt_render")
        return self.rgb, self.ids

    def read_stats(self) -> dict:
        return stats_dict(self.stats)


class BatchRenderer:
    """Many scenes in one batched wavefront (rt_render_batch): one queue, one graph."""

    def __init__(self, scenes: Sequence[Scene], cameras, params, device="cuda", with_ids=True, queue_factor=0.0,
                 queue_chunk=0, graph=True, per_sample=False, tile=0):
        import torch
        n = len(scenes)
        assert n == len(cameras) == len(params) and n > 0
        for s in scenes:
            if s.blob is None:
                s.upload(device)
        self.scenes, self.cameras, self.params = list(scenes), list(cameras), list(params)
        self.device, self.graph = device, graph
        self.base_flags = FLAG_PER_SAMPLE if per_sample else 0
        self.queue_factor, self.queue_chunk = queue_factor, queue_chunk
        self._h = (C.c_void_p * n)(*[s.handle.value for s in scenes])
        self._cams = (CameraC * n)(*[camera_c(c) for c in cameras])
        tiles = list(tile) if isinstance(tile, (list, tuple)) else [tile] * n
        self._params = (ParamsC * n)(*[params_c(p, self.base_flags, 0, queue_factor, queue_chunk, t)
                                       for p, t in zip(params, tiles)])
        nb = lib().rt_render_batch_workspace_bytes(self._h, self._cams, self._params, n)
        if nb == 0:
            raise RTError(-1, "rt_render_batch_workspace_bytes", lib().rt_last_error().decode())
        self.ws_bytes = int(nb)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.rgb, self.ids = [], []
        for c, p in zip(cameras, params):
            shape = (c.height, c.width, p.spp, 3) if per_sample else (c.height, c.width, 3)
            self.rgb.append(torch.empty(shape, dtype=torch.float32, device=device))
            self.ids.append(torch.empty((c.height, c.width, p.spp), dtype=torch.int32, device=device)
                            if with_ids else None)
        self._rgb_p = (C.c_void_p * n)(*[t.data_ptr() for t in self.rgb])
        self._ids_p = (C.c_void_p * n)(*[(t.data_ptr() if t is not None else None) for t in self.ids])
        self.stats = torch.zeros(C.sizeof(Stats) + 64, dtype=torch.uint8, device=device)

    def render(self, flags=0, stream=None, reset_stats=True):
        if reset_stats:
            self.stats.zero_()
        if not self.graph:
            flags |= FLAG_NO_GRAPH
        p0 = self._params[0]
        p0.flags = flags | self.base_flags | (FLAG_GI if getattr(self.params[0], "gi", 0) else 0)
        p0.workspace, p0.workspace_bytes = self.ws.data_ptr(), self.ws_bytes
        p0.stats = self.stats.data_ptr()
        p0.stream = _stream_ptr(stream)
        _check(lib().rt_render_batch(self._h, self._cams, self._params, len(self.scenes), self._rgb_p, self._ids_p),
               "rt_render_batch")
        return self.rgb, self.ids

    def read_stats(self) -> dict:
        return stats_dict(self.stats)


def render(scene: Scene, camera, params, flags=FLAG_SYNC, **kw):
    """One frame: returns (rgb [H,W,3] f32, ids [H,W,spp] i32, stats dict) as torch device tensors."""
    r = Renderer(scene, camera, params, **kw)
    rgb, ids = r.render(flags)
    st = r.read_stats()
    if st["status"]:
        raise RTError(-5, "rt_render", f"queue overflow (status {st['status']}); raise queue_factor")
    return rgb, ids, st


def _trace(scene: Scene, rays, any_hit: bool, stream=None, want_uv: bool = False):
    import torch
    if scene.blob is None:
        scene.upload()
    rays = rays.to(device=scene.blob.device, dtype=torch.float32).contiguous().reshape(-1, 8)
    n = rays.shape[0]
    ws = torch.zeros(256, dtype=torch.uint8, device=rays.device)
    L = lib()
    if any_hit:
        occ = torch.empty(n, dtype=torch.uint8, device=rays.device)
        _check(L.rt_occluded(scene.handle, rays.data_ptr(), n, occ.data_ptr(), ws.data_ptr(), _stream_ptr(stream)),
               "rt_occluded")
        return occ
    t = torch.empty(n, dtype=torch.float32, device=rays.device)
    ids = torch.empty(n, dtype=torch.int32, device=rays.device)
    uv = torch.empty((n, 2), dtype=torch.float32, device=rays.device) if want_uv else None
    _check(L.rt_intersect(scene.handle, rays.data_ptr(), n, t.data_ptr(), ids.data_ptr(),
                          uv.data_ptr() if want_uv else None, ws.data_ptr(), _stream_ptr(stream)), "rt_intersect")
    return (t, ids, uv) if want_uv else (t, ids)


def intersect(scene: Scene, rays, stream=None, uv: bool = False):
    """Closest hit of device rays [n,8] (o, d, tmin, tmax) -> (t [n], id [n]) device tensors, and with
    uv=True also the hit's surface coordinates [n,2] (triangle barycentrics of v1 and v2, sphere
    longitude and polar angle of the normal over 2 pi and pi, 0 for planes and misses)."""
    return _trace(scene, rays, False, stream, uv)


def occluded(scene: Scene, rays, stream=None):
    """Any hit in (0, tmax) of device rays [n,8] -> uint8 [n] device tensor."""
    return _trace(scene, rays, True, stream)


def kernel_times(reset: bool = True) -> dict:
    """Totals recorded by frames rendered with FLAG_TIME_KERNELS (every traversal and shading launch) or
    FLAG_TIME_SHADOW (the shadow launches only): {kernel: (ms, launches)}."""
    ms = (C.c_double * 5)()
    n = (C.c_int64 * 5)()
    _check(lib().rt_kernel_times(ms, n, int(reset)), "rt_kernel_times")
    return {k: (ms[i], n[i]) for i, k in enumerate(("extend", "shade", "shadow", "cache_infer", "cache_train"))}


def make_rays(o, d, tmax=None) -> np.ndarray:
    """Pack origins/directions into the [n,8] FP32 ray layout (tmin column unused)."""
    o = np.asarray(o, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64).reshape(-1, 3)
    R = np.zeros((len(o), 8), np.float32)
    R[:, 0:3] = o
    R[:, 3:6] = d
    if tmax is not None:
        R[:, 7] = np.broadcast_to(np.asarray(tmax, np.float64), (len(o),))
    return R


# ---------------------------------------------------------------------------- radiance-cache network

def bf16_bits(t):
    """float32 tensor -> BF16 bit patterns (round to nearest even) as int16 tensor (same device)."""
    import torch
    return t.to(torch.bfloat16).view(torch.int16)


def bf16_to_f32(bits):
    import torch
    return bits.view(torch.bfloat16).to(torch.float32)


def mlp_num_params() -> int:
    return int(lib().rt_mlp_num_params())


def mlp_forward(w_bf16, x_bf16, stream=None):
    """y [n,3] f32 for features x_bf16 [n,64] (int16 BF16 bits) and weights w_bf16 [num_params]."""
    import torch
    n = x_bf16.shape[0]
    y = torch.empty((n, 3), dtype=torch.float32, device=x_bf16.device)
    _check(lib().rt_mlp_forward(w_bf16.data_ptr(), x_bf16.data_ptr(), n, y.data_ptr(), _stream_ptr(stream)),
           "rt_mlp_forward")
    return y


def mlp_grad(w_bf16, x_bf16, target, dw, loss_sum, n_total=None, stream=None):
    n = x_bf16.shape[0]
    _check(lib().rt_mlp_grad(w_bf16.data_ptr(), x_bf16.data_ptr(), target.data_ptr(), n, n_total or n,
                             dw.data_ptr(), loss_sum.data_ptr(), _stream_ptr(stream)), "rt_mlp_grad")


def mlp_adam(w, w_bf16, m, v, grad, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    _check(lib().rt_mlp_adam(w.data_ptr(), w_bf16.data_ptr(), m.data_ptr(), v.data_ptr(), grad.data_ptr(), int(step),
                             lr, b1, b2, eps, _stream_ptr(stream)), "rt_mlp_adam")


class RadianceCache:
    """Device state of the learned form: weights, Adam moments, last frame's training batch."""

    def __init__(self, weights, capacity: int = 65536, device="cuda"):
        import torch
        L = CacheLayout()
        _check(lib().rt_cache_state_layout(int(capacity), C.byref(L)), "rt_cache_state_layout")
        self.layout = {k: int(getattr(L, k)) for k, _ in CacheLayout._fields_}
        self.capacity = int(capacity)
        self._buf = torch.empty(self.layout["total"] + 256, dtype=torch.uint8, device=device)
        self.base = (self._buf.data_ptr() + 255) // 256 * 256
        self._off = self.base - self._buf.data_ptr()
        w = np.ascontiguousarray(np.concatenate([np.asarray(x, np.float32).reshape(-1) for x in weights])
                                 if isinstance(weights, (list, tuple)) else np.asarray(weights, np.float32))
        assert w.size == mlp_num_params(), w.size
        _check(lib().rt_cache_init(self.base, self.capacity, w.ctypes.data, _stream_ptr()), "rt_cache_init")

    def _view(self, key, nbytes, dtype):
        import torch
        o = self._off + self.layout[key]
        return self._buf[o:o + nbytes].view(dtype)

    def master_weights(self):
        import torch
        return self._view("w_master", 4 * mlp_num_params(), torch.float32).clone()

    def bf16_weights(self):
        import torch
        return self._view("w_bf16", 2 * mlp_num_params(), torch.int16).clone()

    def counters(self) -> dict:
        import torch
        c = self._view("counters", 256, torch.int32).cpu().numpy()
        return {"steps": int(c[0]), "n_train": int(c[1]), "loss_sums": c[2:18].view(np.float32).copy(),
                "health": int(c[18])}

    def health(self) -> int:
        """CACHE_HEALTH_* bits of the state (0: healthy; set bits make learned-form frames fall back to the
        plain tracer until the state is initialised again)."""
        return self.counters()["health"]

    def save(self, path: str) -> None:
        """Checkpoint of the network: FP32 master weights, Adam moments and the step count (an .npz file)."""
        import torch
        n = mlp_num_params()
        torch.cuda.synchronize()
        np.savez(path, format=np.array("mirt-radiance-cache-1"), capacity=np.array(self.capacity),
                 w_master=self._view("w_master", 4 * n, torch.float32).cpu().numpy(),
                 m=self._view("m", 4 * n, torch.float32).cpu().numpy(),
                 v=self._view("v", 4 * n, torch.float32).cpu().numpy(),
                 steps=np.array(self.counters()["steps"], np.int64))

    @staticmethod
    def read_checkpoint(path: str) -> dict:
        """Validated arrays of a checkpoint written by save() (no device work)."""
        n = mlp_num_params()
        with np.load(path, allow_pickle=False) as z:
            if "format" not in z.files or str(z["format"]) != "mirt-radiance-cache-1":
                raise ValueError(f"{path}: not a radiance-cache checkpoint")
            ck = {k: z[k] for k in ("w_master", "m", "v", "steps", "capacity")}
        for k in ("w_master", "m", "v"):
            a = ck[k]
            if a.dtype != np.float32 or a.shape != (n,):
                raise ValueError(f"{path}: {k} must be float32 [{n}], got {a.dtype} {a.shape}")
            if not np.isfinite(a).all():
                raise ValueError(f"{path}: {k} holds non-finite values")
        if (ck["v"] < 0).any() or int(ck["steps"]) < 0:
            raise ValueError(f"{path}: negative second moment or step count")
        return ck

    @classmethod
    def load(cls, path: str, capacity: int = None, device="cuda") -> "RadianceCache":
        """A state restored from save(): master weights (and their BF16 copy), Adam moments, step count."""
        import torch
        ck = cls.read_checkpoint(path)
        cache = cls(ck["w_master"], capacity=int(capacity or ck["capacity"]), device=device)
        n = mlp_num_params()
        cache._view("m", 4 * n, torch.float32).copy_(torch.from_numpy(ck["m"]))
        cache._view("v", 4 * n, torch.float32).copy_(torch.from_numpy(ck["v"]))
        cache._view("counters", 4, torch.int32).fill_(int(ck["steps"]))
        torch.cuda.synchronize()
        return cache

    def training_batch(self):
        """(rays [n,6], features [n,64] f32, targets [n,3], pixel [n]) of the last trained frame (device tensors)."""
        import torch
        n = self.counters()["n_train"]
        rays = self._view("train_rays", 24 * self.capacity, torch.float32).reshape(-1, 6)[:n]
        feats = self._view("train_feats", 128 * self.capacity, torch.int16).reshape(-1, 64)[:n]
        tg = self._view("train_targets", 12 * self.capacity, torch.float32).reshape(-1, 3)[:n]
        pix = self._view("train_pix", 4 * self.capacity, torch.int32)[:n]
        return rays.clone(), bf16_to_f32(feats.contiguous()), tg.clone(), pix.clone()


class CachedRenderer(Renderer):
    """Frames of the learned form: recursion below `depth` answered (and trained) by the network."""

    def __init__(self, scene: Scene, camera, params, cache: RadianceCache, mode=CACHE_TRAIN, depth=2, full_depth=8,
                 train_samples=None, train_steps=4, lr=1e-3, bounds=None, **kw):
        self.cache = cache
        self.cc = CacheC()
        self.cc.mode, self.cc.depth, self.cc.full_depth = int(mode), int(depth), int(full_depth)
        self.cc.train_samples = int(train_samples or cache.capacity)
        self.cc.train_steps = int(train_steps)
        self.cc.lr, self.cc.b1, self.cc.b2, self.cc.eps = float(lr), 0.9, 0.999, 1e-8
        if bounds is not None:
            self.cc.bounds_lo[:] = [float(x) for x in bounds[0]]
            self.cc.bounds_hi[:] = [float(x) for x in bounds[1]]
        self.cc.state = cache.base
        super().__init__(scene, camera, params, **kw)

    def _alloc(self, with_ids):
        import torch
        p = params_c(self.params, self.base_flags, self.samples_per_pass, self.queue_factor, self.queue_chunk, self.tile)
        n = lib().rt_render_cached_workspace_bytes(self.scene.handle, C.byref(self.cam_c), C.byref(p),
                                                   C.byref(self.cc))
        if n == 0:
            raise RTError(-1, "rt_render_cached_workspace_bytes", lib().rt_last_error().decode())
        self.ws_bytes = int(n)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        H, W = self.camera.height, self.camera.width
        shape = (H, W, self.params.spp, 3) if self.base_flags & FLAG_PER_SAMPLE else (H, W, 3)
        self.rgb = torch.empty(shape, dtype=torch.float32, device=self.device)
        self.ids = torch.empty((H, W, self.params.spp), dtype=torch.int32, device=self.device) if with_ids else None
        self.stats = torch.zeros(C.sizeof(Stats) + 64, dtype=torch.uint8, device=self.device)

    def set_mode(self, mode):
        self.cc.mode = int(mode)

    def render(self, flags=0, stream=None, reset_stats=True):
        if reset_stats:
            self.stats.zero_()
        if not self.graph:
            flags |= FLAG_NO_GRAPH
        p = params_c(self.params, flags | self.base_flags, self.samples_per_pass, self.queue_factor,
                     self.queue_chunk, self.tile)
        p.workspace, p.workspace_bytes = self.ws.data_ptr(), self.ws_bytes
        p.stats = self.stats.data_ptr()
        p.stream = _stream_ptr(stream)
        _check(lib().rt_render_cached(self.scene.handle, C.byref(self.cam_c), C.byref(p), C.byref(self.cc),
                                      self.rgb.data_ptr(), _ptr(self.ids)), "rt_render_cached")
        return self.rgb, self.ids
