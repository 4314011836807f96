"""Autotuner for the wavefront tracer: primary-ray tile, queue chunk and BVH node layout.

The three knobs change only where work sits in memory and how it is handed out
to waves, never what is computed: the tile shape decides which 64 pixels share
a wave (and so how coherent the secondary rays of a wave are), the queue chunk
how many queue entries a persistent traversal wave takes per atomic fetch, and
the node layout (binary tree depth-first, breadth-first or in three-level
treelets, or its four-wide collapse with float or 8-bit quantized child boxes)
which nodes share cache lines and how many bytes and dependent node fetches a
ray needs.  The tuner times real frames of the caller's workload
through the C-ABI, keeps the fastest setting, and checks that every candidate
returns the same primary-hit ids as the default setting (a candidate that
does not is rejected).

Search: coordinate descent from the defaults (8x8, 128, depth-first) over
layout, then chunk, then tile, repeated until a sweep changes nothing (at most
`rounds` sweeps).  Results may be cached in a JSON file keyed by the device
name and a signature of the workload.
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
from typing import Callable, Optional, Sequence

from . import rt

SPACE = {
    "layout": [rt.LAYOUT_DFS, rt.LAYOUT_BFS, rt.LAYOUT_TREELET, rt.LAYOUT_BVH4, rt.LAYOUT_BVH4Q],
    "chunk": [64, 128, 256, 512, 1024],
    "tile": [rt.TILE_8X8, rt.TILE_16X4, rt.TILE_32X2, rt.TILE_4X16],
}
DEFAULT = {"layout": rt.LAYOUT_DFS, "chunk": 128, "tile": rt.TILE_8X8}


def signature(scenes: Sequence["rt.Scene"], cameras, params) -> str:
    """Stable description of a workload: primitive counts, resolutions, samples, depths and path tracing."""
    h = hashlib.sha256()
    for s, c, p in zip(scenes, cameras, params):
        h.update(f"{len(s.src.spheres)},{len(s.src.tris)},{len(s.src.planes)},{len(s.src.lights)};"
                 f"{c.width}x{c.height};{p.spp},{p.max_depth},{int(getattr(p, 'gi', 0))};".encode())
    return h.hexdigest()[:16]


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"


class _Workload:
    """Renders the workload with a given setting and times it on the current stream."""

    def __init__(self, scenes, cameras, params, batch: bool):
        self.scenes, self.cameras, self.params = list(scenes), list(cameras), list(params)
        self.batch = batch
        self.layout = None

    def _set_layout(self, layout):
        if layout == self.layout:
            return
        for s in self.scenes:
            if s.info["node_layout"] != layout:
                s.set_layout(layout)
            if s.blob is None:
                s.upload()
        self.layout = layout

    def run(self, cfg, warmup: int, steps: int):
        """(median ms per frame, primary-hit ids of every scene as host arrays)."""
        import torch
        self._set_layout(cfg["layout"])
        if self.batch:
            r = rt.BatchRenderer(self.scenes, self.cameras, self.params, queue_chunk=cfg["chunk"], tile=cfg["tile"])
            frame = r.render
        else:
            rs = [rt.Renderer(s, c, p, queue_chunk=cfg["chunk"], tile=cfg["tile"])
                  for s, c, p in zip(self.scenes, self.cameras, self.params)]

            def frame():
                for x in rs:
                    x.render()
        frame()
        torch.cuda.synchronize()
        st = r.read_stats() if self.batch else rs[0].read_stats()
        if st["status"]:
            raise rt.RTError(-5, "autotune", f"queue overflow with {cfg}")
        ids = [t.cpu().numpy().copy() for t in (r.ids if self.batch else [x.ids for x in rs])]
        for _ in range(warmup):
            frame()
        ms = []
        for _ in range(steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            frame()
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return statistics.median(ms), ids


def tune(scenes: Sequence["rt.Scene"], cameras, params, batch: bool = True, warmup: int = 1, steps: int = 3,
         rounds: int = 2, space: Optional[dict] = None, cache_path: Optional[str] = None,
         log: Optional[Callable[[str], None]] = None) -> dict:
    """Pick {layout, chunk, tile} for the workload; leaves every scene in the chosen layout, uploaded.

    Returns {"config": {...}, "ms": best median ms, "default_ms": ms of the defaults, "trials": [...],
    "key": cache key, "cached": bool}.
    """
    import numpy as np
    space = space or SPACE
    key = f"{_device_name()}|{'batch' if batch else 'seq'}|{signature(scenes, cameras, params)}"
    if cache_path:
        hit = read_cache(cache_path, key, log)
        if hit is not None:
            res = dict(hit, cached=True)
            _Workload(scenes, cameras, params, batch)._set_layout(res["config"]["layout"])
            return res
    W = _Workload(scenes, cameras, params, batch)
    trials = []
    seen = {}

    def measure(cfg):
        k = (cfg["layout"], cfg["chunk"], cfg["tile"])
        if k not in seen:
            ms, ids = W.run(cfg, warmup, steps)
            ok = ref_ids is None or all(np.array_equal(a, b) for a, b in zip(ids, ref_ids))
            seen[k] = ms if ok else float("inf")
            trials.append({"config": dict(cfg), "ms": round(ms, 4), "ids_match": ok})
            if log:
                log(f"autotune {cfg}: {ms:.3f} ms{'' if ok else ' (ids differ: rejected)'}")
        return seen[k]

    ref_ids = None
    best = dict(DEFAULT)
    _, ref_ids = W.run(best, 0, 1)
    best_ms = default_ms = measure(best)
    for _ in range(max(1, rounds)):
        changed = False
        for dim in ("layout", "chunk", "tile"):
            for v in space[dim]:
                cand = dict(best, **{dim: v})
                ms = measure(cand)
                if ms < best_ms * 0.995:     # ignore sub-noise gains
                    best, best_ms, changed = cand, ms, True
        if not changed:
            break
    W._set_layout(best["layout"])
    res = {"config": best, "ms": round(best_ms, 4), "default_ms": round(default_ms, 4), "trials": trials,
           "key": key, "cached": False}
    if cache_path:
        write_cache(cache_path, key, {k: v for k, v in res.items() if k != "cached"})
    return res


def _load_db(path: str, log: Optional[Callable[[str], None]] = None) -> dict:
    """The cache file as a dict; an unreadable or malformed file counts as empty (and is reported)."""
    if not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError) as e:
        if log:
            log(f"autotune cache {path} unreadable ({e.__class__.__name__}): using defaults and tuning afresh")
        return {}
    if not isinstance(db, dict):
        if log:
            log(f"autotune cache {path} is not a JSON object: ignored")
        return {}
    return db


def _valid_entry(e) -> bool:
    if not isinstance(e, dict) or not isinstance(e.get("config"), dict):
        return False
    cfg = e["config"]
    return (set(cfg) == set(SPACE) and all(isinstance(cfg[k], int) and cfg[k] in SPACE[k] for k in SPACE)
            and isinstance(e.get("ms"), (int, float)))


def read_cache(path: str, key: str, log: Optional[Callable[[str], None]] = None) -> Optional[dict]:
    """The cached result for key, or None when the file is missing, corrupt, or its entry is malformed
    (a setting outside the search space is never applied: the caller tunes afresh)."""
    e = _load_db(path, log).get(key)
    if e is None:
        return None
    if not _valid_entry(e):
        if log:
            log(f"autotune cache entry {key} malformed: ignored")
        return None
    return e


def write_cache(path: str, key: str, entry: dict) -> None:
    """Add or replace one entry; the file is replaced atomically, so a crash never leaves half a file."""
    db = _load_db(path)
    db[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1)
    os.replace(tmp, path)
