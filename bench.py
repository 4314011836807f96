#!/usr/bin/env python3
"""Benchmark: Mrays/s and ms/frame of the Whitted tracer on one MI355X.

Workload (default "c2"): 1920x1080 at 16 jittered spp, 1,000 icospheres
(1.28M triangles), 50% Phong / 30% mirror / 20% glass, 8 point lights, max
depth 8 -- the plain depth-8 tracer.  One step = one full frame (every
wavefront pass, bounce and shadow query).  Inputs (scene blob) are resident in
HBM before the timed region.

Prints ONE JSON line.  roofline: the dominant traversal kernel's algorithmic
bytes (64 B per BVH node fetched + 48 B per triangle record + 32 B per sphere,
counted by an untimed counting frame) divided by its average launch time from
HIP events recorded on the launch stream during the timed frames.
cpu_baseline: the FP64 brute-force oracle on a bounded pixel sample of the
same frame, on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    from paper_1504_03151_amd import scenes
    if name == "c0":
        return scenes.config0()
    if name == "c1":
        return scenes.config1()
    if name == "c2":
        return scenes.config2()
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(w, budget_s: float, seed: int = 5):
    import numpy as np

    import oracle
    from paper_1504_03151_amd import scenes
    ncores = len(os.sched_getaffinity(0))
    pix = scenes.pixel_subset(w.camera, 1 << 20, seed)
    done, rays, elapsed, n = 0, 0, 0.0, 4
    while elapsed < budget_s and done < len(pix):
        chunk = pix[done:done + n]
        t0 = time.perf_counter()
        out = oracle.render(w.scene, w.camera, w.params, chunk, nthreads=ncores)
        dt = time.perf_counter() - t0
        elapsed += dt
        rays += int(out["counts"].sum())
        done += len(chunk)
        per_px = dt / max(1, len(chunk))
        n = int(min(max(4, (budget_s - elapsed) / max(per_px, 1e-6) * 0.8), 4096))
    return {"value": rays / elapsed / 1e6, "unit": "Mrays/s", "cores": ncores, "kind": "oracle",
            "sample": f"{done} seeded pixels x {w.params.spp} spp of the same frame ({rays} rays, "
                      f"{elapsed:.1f} s, FP64 brute force over every primitive, no BVH)"}


def build_scenes(ws, rt, threads=16):
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda w: rt.Scene(w.scene), ws))


def bench_batch(args):
    """256 uneven scenes: one batched wavefront vs 256 sequential single-scene frames."""
    import torch
    from paper_1504_03151_amd import rt, scenes
    t0 = time.perf_counter()
    ws = scenes.config3(args.n_scenes)
    log(f"generated {len(ws)} scenes in {time.perf_counter() - t0:.1f} s: "
        f"{sum(len(w.scene.tris) for w in ws)} triangles, {sum(w.camera.n_pixels for w in ws)} pixels")
    t0 = time.perf_counter()
    scs = build_scenes(ws, rt)
    log(f"built {len(scs)} BVHs in {time.perf_counter() - t0:.1f} s")
    for sc in scs:
        sc.upload()
    br = rt.BatchRenderer(scs, [w.camera for w in ws], [w.params for w in ws], queue_chunk=args.queue_chunk)
    log(f"batch workspace {br.ws_bytes / 2 ** 30:.2f} GiB")
    br.render(rt.FLAG_SYNC)
    st = br.read_stats()
    assert st["status"] == 0, st
    rays, shadow = sum(st["rays"]), sum(st["shadow"])
    for _ in range(args.warmup):
        br.render()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        br.render()
    torch.cuda.synchronize()
    batched_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # sequential baseline: one single-scene frame after another on the same stream (graphs cached)
    rs = [rt.Renderer(sc, w.camera, w.params, queue_chunk=args.queue_chunk) for sc, w in zip(scs, ws)]
    for r in rs:
        r.render()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for r in rs:
            r.render()
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    value = (rays + shadow) / (batched_ms / 1e3) / 1e6
    log(f"batched {batched_ms:.2f} ms, sequential {seq_ms:.2f} ms ({seq_ms / batched_ms:.2f}x), {value:.0f} Mrays/s")
    print(json.dumps({
        "metric": "Mrays/s of one batched frame of 256 uneven scenes", "value": round(value, 2), "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(batched_ms, 3),
        "sequential_ms": round(seq_ms, 3), "speedup_vs_sequential": round(seq_ms / batched_ms, 3),
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c3_batch_{len(ws)}_scenes", "rays": rays, "shadow_rays": shadow,
                   "triangles": sum(len(w.scene.tris) for w in ws),
                   "pixels": sum(w.camera.n_pixels for w in ws)}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--graph", action="store_true", help="time graph replays (no per-kernel events)")
    ap.add_argument("--samples-per-pass", type=int, default=0, help="0 = chosen by the library")
    ap.add_argument("--queue-chunk", type=int, default=0, help="0 = library default")
    ap.add_argument("--n-scenes", type=int, default=256, help="scenes of the c3 batch")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); the path would shard "
              f"pixels or sample passes across GPUs, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1504_03151_amd import rt
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    rt.lib()
    if args.workload == "c3":
        return bench_batch(args)
    w = workload(args.workload)
    log(f"workload {w.name}: {len(w.scene.spheres)} spheres, {len(w.scene.tris)} triangles, "
        f"{len(w.scene.planes)} planes, {len(w.scene.lights)} lights")
    t0 = time.perf_counter()
    sc = rt.Scene(w.scene)
    log(f"BVH build {time.perf_counter() - t0:.2f} s: {sc.info}")
    sc.upload()
    r = rt.Renderer(sc, w.camera, w.params, samples_per_pass=args.samples_per_pass, queue_chunk=args.queue_chunk)
    log(f"workspace {r.ws_bytes / 2 ** 30:.2f} GiB")

    # untimed counting frame: rays per depth and BVH work of every traversal launch
    r.render(rt.FLAG_COUNT_WORK | rt.FLAG_SYNC | rt.FLAG_NO_GRAPH)
    cst = r.read_stats()
    assert cst["status"] == 0, cst
    rays = sum(cst["rays"])
    shadow = sum(cst["shadow"])
    log(f"rays/frame {rays} closest-hit + {shadow} shadow; passes {cst['passes']}")

    flags = 0 if args.graph else rt.FLAG_TIME_KERNELS
    for _ in range(args.warmup):
        r.render(flags)
    torch.cuda.synchronize()
    rt.kernel_times(reset=True)
    log("timing")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r.render(flags)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = rt.kernel_times(reset=True)
    st = r.read_stats()
    assert st["status"] == 0, st
    ms = (t1 - t0) * 1e3 / args.steps
    value = (rays + shadow) / (ms / 1e3) / 1e6
    log(f"{ms:.2f} ms/frame, {value:.1f} Mrays/s; kernel ms {kt}")

    roof = None
    if not args.graph:
        per = {
            "extend": 64 * cst["node_visits"] + 48 * cst["tri_tests"] + 32 * cst["sphere_tests"],
            "shadow": 64 * cst["shadow_node_visits"] + 48 * cst["shadow_tri_tests"] + 32 * cst["shadow_sphere_tests"],
        }
        dom = max(("extend", "shadow"), key=lambda k: kt[k][0])
        launches_per_frame = kt[dom][1] / args.steps
        avg_launch_s = kt[dom][0] / 1e3 / kt[dom][1]
        bytes_per_launch = per[dom] / launches_per_frame
        achieved = bytes_per_launch / avg_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": f"k_{dom}",
                "avg_launch_ms": round(avg_launch_s * 1e3, 4), "bytes_per_launch": int(bytes_per_launch),
                "kernel_ms_per_frame": {k: round(v[0] / args.steps, 3) for k, v in kt.items()}}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(w, args.cpu_seconds)

    out = {
        "metric": "Mrays/s (closest-hit + shadow rays per second), plain depth-8 Whitted frame",
        "value": round(value, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "ms_per_frame": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "width": w.camera.width, "height": w.camera.height, "spp": w.params.spp,
                   "max_depth": w.params.max_depth, "triangles": len(w.scene.tris),
                   "spheres": len(w.scene.spheres), "lights": len(w.scene.lights),
                   "rays_per_frame": rays, "shadow_rays_per_frame": shadow, "parallelism": "single-gpu"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
