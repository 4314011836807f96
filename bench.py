#!/usr/bin/env python3
"""Benchmark: Mrays/s and ms/frame of the Whitted tracer on one MI355X.

Workload (default "c2"): 1920x1080 at 16 jittered spp, 1,000 icospheres
(1.28M triangles), 50% Phong / 30% mirror / 20% glass, 8 point lights, max
depth 8 -- the plain depth-8 tracer.  One step = one full frame (every
wavefront pass, bounce and shadow query).  Inputs (scene blob) are resident in
HBM before the timed region.

Prints ONE JSON line.  roofline: the dominant traversal kernel's algorithmic
bytes (64 B per binary or quantized four-wide node fetched, 128 B per float
four-wide node, + 48 B per triangle record + 32 B per sphere, counted by an
untimed counting frame) divided by its average launch time from HIP events
recorded on the launch stream during the timed frames.
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
# FP32 vector peak 157.3 TFLOP/s = 256 CUs x 2.4 GHz x 128 lanes x 2 (FMA): two wave64 VALU instructions per
# CU per clock (the traversal kernels issue 1.3 per CU-clock, so one per clock is not the limit)
VALU_PEAK_WAVE_INSTS = 256 * 2.4e9 * 2
VALU_PEAK_LANE_OPS = VALU_PEAK_WAVE_INSTS * 64


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name, area_radius=0.0):
    from paper_1504_03151_amd import scenes
    if name == "c0":
        w = scenes.config0()
    elif name == "c1":
        w = scenes.config1()
    elif name == "c2":
        w = scenes.config2()
    elif name == "gi":
        w = scenes.config_gi()
    else:
        raise SystemExit(f"unknown workload {name}")
    if area_radius > 0.0:
        w = scenes.with_disk_lights(w, area_radius)
    return w


def cpu_baseline(w, budget_s: float, seed: int = 5, scene=None):
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
    out = {"value": rays / elapsed / 1e6, "unit": "Mrays/s", "cores": ncores, "kind": "oracle",
           "sample": f"{done} seeded pixels x {w.params.spp} spp of the same frame ({rays} rays, "
                     f"{elapsed:.1f} s, FP64 brute force over every primitive, no BVH)"}
    if scene is not None:
        # the fair CPU figure beside it: the library's FP32 host traversal of the same BVH on the camera rays
        # of the same pixels (closest hit only), all host cores
        from paper_1504_03151_amd import rt
        from paper_1504_03151_amd import scenes
        o, d = oracle.camera_rays(w.camera, w.params, scenes.pixel_subset(w.camera, 1 << 18, seed))
        R = rt.make_rays(o, d)
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < 2.0 or reps == 0:
            scene.host_trace(R, nthreads=ncores)
            reps += 1
        dt = time.perf_counter() - t0
        out["host_bvh"] = {"value": round(reps * len(R) / dt / 1e6, 3), "unit": "Mrays/s", "cores": ncores,
                           "sample": f"{len(R)} camera rays of seeded pixels of the same frame, closest hit, FP32 "
                                     f"BVH traversal on the host (layout {scene.info['node_layout']}), {reps} runs"}
    return out


KERNEL_SOURCES = ["paper_1504_03151_amd/csrc/rt_common.h", "paper_1504_03151_amd/csrc/render.cpp"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_record(kind, kernel, workload, tile, layout, chunk):
    """The `kind` record ("traffic-record": HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE;
    "valu-record": VALU work per launch from the SQ counters) of this kernel, workload and setting in the
    committed profile summaries; None when none matches or the kernel sources changed since."""
    import glob
    want = {"kernel": kernel, "workload": workload, "tile": tile, "layout": layout, "queue_chunk": chunk,
            "source_sha256_16": kernel_source_hash()}
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(f) as fh:
            for line in fh:
                if line.startswith(kind + ":"):
                    try:
                        rec = json.loads(line.split(":", 1)[1])
                    except ValueError:
                        continue
                    if all(rec.get(k) == v for k, v in want.items()):
                        return rec
    return None


def traffic_record(kernel, workload, tile, layout, chunk):
    rec = profile_record("traffic-record", kernel, workload, tile, layout, chunk)
    return None if rec is None else int(rec["bytes_per_launch"])


def bench_progressive(args):
    """Progressive rendering, the shape of the paper's pass-by-pass experiment (Section V, Fig. 5-6): every pass
    samples each area light once and adds into the accumulator.  Reports passes per second (graph replays) and
    the relative MSE of the running average after 1, 4, 16, 64 and 256 passes against a 1024-pass average."""
    import numpy as np
    import torch
    from paper_1504_03151_amd import rt
    w = workload(args.workload, args.area_lights or 2.0)
    w.params.spp, w.params.jitter = 1, 1
    sc = rt.Scene(w.scene, node_layout=rt.LAYOUT_BVH4Q).upload()
    r = rt.Renderer(sc, w.camera, w.params, with_ids=False)
    ref_passes = 1024
    for f in range(ref_passes):
        w.params.frame = f
        img, _ = r.render(accum_frames=f)
    torch.cuda.synchronize()
    ref = img.clone().double()

    def rel_mse(x):
        return float(((x.double() - ref) ** 2 / (ref ** 2 + 0.01)).mean())

    curve = {}
    for f in range(256):
        w.params.frame = 100000 + f
        img, _ = r.render(accum_frames=f)
        if f + 1 in (1, 4, 16, 64, 256):
            torch.cuda.synchronize()
            curve[str(f + 1)] = rel_mse(img)
    n = max(args.steps, 64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(n):
        w.params.frame = 200000 + f
        r.render(accum_frames=f)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = r.read_stats()
    assert st["status"] == 0, st
    rays = sum(st["rays"]) + sum(st["shadow"])
    log(f"progressive {w.name}: {n / dt:.1f} passes/s, rel-MSE vs {ref_passes} passes {curve}")
    print(json.dumps({
        "metric": "passes/s of progressive rendering with area lights sampled once per pass", "value": round(n / dt, 2),
        "unit": "passes/s", "n_gpus": 1, "steps": n, "warmup": ref_passes + 256, "ms_per_step": round(dt * 1e3 / n, 4),
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "mrays_per_s": round(rays / (dt / n) / 1e6, 1), "rel_mse_vs_passes": curve,
        "config": {"workload": w.name, "width": w.camera.width, "height": w.camera.height, "spp_per_pass": 1,
                   "max_depth": w.params.max_depth, "lights": len(w.scene.lights), "reference_passes": ref_passes}}),
          flush=True)


def fixed_config(args) -> bool:
    """Tile, queue chunk and node layout all given on the command line: nothing to tune."""
    return args.tile is not None and args.layout is not None and args.queue_chunk > 0


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
    cams, ps = [w.camera for w in ws], [w.params for w in ws]
    chunk, tile, tuned = args.queue_chunk, args.tile or 0, None
    if args.layout:
        for sc in scs:
            sc.set_layout(args.layout).upload()
    if not (args.no_autotune or fixed_config(args)):
        from paper_1504_03151_amd import autotune
        t0 = time.perf_counter()
        tuned = autotune.tune(scs, cams, ps, batch=True, log=log)
        chunk, tile = tuned["config"]["chunk"], tuned["config"]["tile"]
        log(f"autotune {time.perf_counter() - t0:.1f} s: {tuned['config']} {tuned['ms']:.3f} ms "
            f"(defaults {tuned['default_ms']:.3f} ms)")
    br = rt.BatchRenderer(scs, cams, ps, queue_chunk=chunk, tile=tile)
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
    rs = [rt.Renderer(sc, w.camera, w.params, queue_chunk=chunk, tile=tile) for sc, w in zip(scs, ws)]
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
        "autotune": None if tuned is None else {"config": tuned["config"], "ms": tuned["ms"],
                                                 "default_ms": tuned["default_ms"], "trials": len(tuned["trials"])},
        "config": {"workload": f"c3_batch_{len(ws)}_scenes", "rays": rays, "shadow_rays": shadow,
                   "triangles": sum(len(w.scene.tris) for w in ws),
                   "pixels": sum(w.camera.n_pixels for w in ws)}}), flush=True)


MFMA_BF16_PEAK_TFLOPS = 2500.0
# algorithmic FLOP of the radiance-cache network (42 real inputs, 4 hidden 64x64 products, 3 outputs)
MLP_FWD_FLOP = 2 * (42 * 64 + 4 * 64 * 64 + 64 * 3)                    # 38,528 per query
MLP_TRAIN_FLOP = MLP_FWD_FLOP + MLP_FWD_FLOP + 2 * (4 * 64 * 64 + 64 * 3)  # forward, dW, input grads: 110,208


def mlp_store_only_tflops(cache, nq, reps=10):
    """Rate of the network alone: rt_mlp_forward (outputs stored, no per-pixel atomic adds) with the cache's
    weights on nq seeded random feature rows in [-1, 1); HIP events around reps launches on the current stream.
    Set beside the cache form's rate it shows what the scatter into the pixels costs."""
    import torch
    from paper_1504_03151_amd import rt
    if nq <= 0:
        return None
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    x = rt.bf16_bits(torch.rand(nq, 64, generator=g, device="cuda") * 2 - 1)
    wb = cache.bf16_weights()
    rt.mlp_forward(wb, x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rt.mlp_forward(wb, x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return nq * MLP_FWD_FLOP / (ms / 1e3) / 1e12


def bench_cache(w, sc, plain, args):
    """Learned form vs the plain full-depth frame on the same scene, camera, samples and frame numbers.

    256 frames of online training (65,536 samples, 4 Adam steps each; 96 for path-traced frames, whose frames
    take ten times longer) warm the network up; the next 16 frames are timed (training included) beside plain
    frames of the same frame numbers, which are the reference of the relative MSE for Whitted frames;
    path-traced frames are compared with a converged mean of plain frames.  The errors after the first 32
    warm-up frames (4 frames, untimed, training as usual) are reported beside.  Depth-2 truncation (the
    network replaced by zero) shows what the network gains.
    """
    import numpy as np
    import torch
    from paper_1504_03151_amd import rt, scenes
    cache = rt.RadianceCache(scenes.mlp_init_weights(2), capacity=65536)
    zero = rt.RadianceCache([np.zeros_like(x) for x in scenes.mlp_init_weights(0)], capacity=1024)
    cr = rt.CachedRenderer(sc, w.camera, w.params, cache, mode=rt.CACHE_TRAIN, depth=2,
                           full_depth=w.params.max_depth, train_samples=65536, train_steps=4, lr=1e-3,
                           queue_chunk=plain.queue_chunk, tile=plain.tile, with_ids=False)
    log(f"cache workspace {cr.ws_bytes / 2 ** 30:.2f} GiB")
    f0 = 1000
    warm = args.cache_warmup if args.cache_warmup is not None else (96 if w.params.gi else 256)
    early = min(32, warm)        # the learned form's own protocol: errors after 32 warm-up frames as well

    def rel_mse(x, ref, mask=None):
        e = (x.double() - ref.double()) ** 2 / (ref.double() ** 2 + 0.01)
        if mask is not None:
            e = e[mask]
        return float(e.mean()) if e.numel() else 0.0

    # Path-traced frames are noisy estimates: their reference is a converged one, the mean of plain frames
    # with other frame numbers (untimed); a single plain frame's own error against it is reported beside.
    ref = None
    if w.params.gi:
        acc = None
        for i in range(args.gi_ref_frames):
            w.params.frame = 50000 + i
            img = plain.render()[0]
            acc = img.double() if acc is None else acc + img.double()
        torch.cuda.synchronize()
        ref = (acc / args.gi_ref_frames).float()
        log(f"reference: mean of {args.gi_ref_frames} plain path-traced frames")

    def timed(renderer):
        # launches one by one with no events inside the frame (each recorded event idles the GPU for a few
        # microseconds); the per-kernel split comes from separate frames below
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        out = renderer.render(rt.FLAG_NO_GRAPH)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b), renderer.read_stats(), out[0]

    def errors_only(first_frame, count):
        """Relative MSE of `count` learned-form frames (training as usual) against plain frames, untimed."""
        out = []
        for f in range(count):
            w.params.frame = first_frame + f
            img_c = cr.render(rt.FLAG_SYNC)[0].clone()
            img_p = plain.render(rt.FLAG_SYNC)[0]
            cr.cc.state, cr.cc.mode = zero.base, rt.CACHE_INFER
            img_t = cr.render(rt.FLAG_SYNC | rt.FLAG_NO_GRAPH)[0]
            cr.cc.state, cr.cc.mode = cache.base, rt.CACHE_TRAIN
            torch.cuda.synchronize()
            aff = ((img_p - img_t).abs() > 1e-6).any(dim=-1)
            target = img_p if ref is None else ref
            out.append({"rel_mse": rel_mse(img_c, target), "rel_mse_affected": rel_mse(img_c, target, aff),
                        "trunc_rel_mse": rel_mse(img_t, target), "trunc_rel_mse_affected": rel_mse(img_t, target, aff)})
        return out

    f = 0
    early_rows = []
    while f < warm:
        w.params.frame = f0 + f
        cr.render()
        f += 1
        if f == early:
            early_rows = errors_only(f0 + f, 4)
            f += 4
            log(f"after {early} warm-up frames: rel-MSE {np.mean([r['rel_mse'] for r in early_rows]):.3e} "
                f"(affected {np.mean([r['rel_mse_affected'] for r in early_rows]):.3e})")
    warm = f
    torch.cuda.synchronize()
    c = cache.counters()
    assert c["health"] == 0, c
    log(f"cache warm-up: {warm} frames, {c['steps']} Adam steps, last loss "
        f"{float(c['loss_sums'][:4].sum()) / (3 * max(1, c['n_train'])):.4f}")

    rows = []
    for f in range(args.cache_frames):
        w.params.frame = f0 + warm + f
        ms_c, st_c, img_c = timed(cr)
        assert st_c["status"] == 0, st_c
        img_c = img_c.clone()
        ms_p, st_p, img_p = timed(plain)
        assert st_p["status"] == 0, st_p
        cr.cc.state, cr.cc.mode = zero.base, rt.CACHE_INFER
        img_t = cr.render(rt.FLAG_SYNC | rt.FLAG_NO_GRAPH)[0]
        cr.cc.state, cr.cc.mode = cache.base, rt.CACHE_TRAIN
        torch.cuda.synchronize()
        aff = ((img_p - img_t).abs() > 1e-6).any(dim=-1)
        target = img_p if ref is None else ref
        rows.append({"ms_cache": ms_c, "ms_plain": ms_p, "rel_mse": rel_mse(img_c, target),
                     "rel_mse_affected": rel_mse(img_c, target, aff), "trunc_rel_mse": rel_mse(img_t, target),
                     "trunc_rel_mse_affected": rel_mse(img_t, target, aff), "affected": float(aff.double().mean()),
                     "plain_rel_mse": rel_mse(img_p, target),
                     "queries": st_c["cache_queries"], "rays": sum(st_c["rays"]) + sum(st_c["shadow"]),
                     "target_rays": st_c["target_rays"] + st_c["target_shadow"],
                     "plain_rays": sum(st_p["rays"]) + sum(st_p["shadow"])})
    n = len(rows)
    # per-kernel split: as many frames of each form again, with events around every launch
    torch.cuda.synchronize()
    rt.kernel_times(reset=True)
    for f in range(n):
        w.params.frame = f0 + warm + n + f
        cr.render(rt.FLAG_TIME_KERNELS)
    torch.cuda.synchronize()
    kt_c = rt.kernel_times(reset=True)
    for f in range(n):
        w.params.frame = f0 + warm + n + f
        plain.render(rt.FLAG_TIME_KERNELS)
    torch.cuda.synchronize()
    kt_p = rt.kernel_times(reset=True)
    med = lambda key: float(np.median([r[key] for r in rows]))
    mean = lambda key: float(np.mean([r[key] for r in rows]))
    ms_c, ms_p = med("ms_cache"), med("ms_plain")
    q = mean("queries")
    inf_ms = kt_c["cache_infer"][0] / n
    tr_ms = kt_c["cache_train"][0] / n
    inf_tflops = q * MLP_FWD_FLOP / (inf_ms / 1e3) / 1e12 if inf_ms > 0 else None
    tr_tflops = 65536 * MLP_TRAIN_FLOP / (tr_ms / 1e3) / 1e12 if tr_ms > 0 else None
    so_tflops = mlp_store_only_tflops(cache, int(q))
    out = {
        "ms_per_frame": round(ms_c, 3), "plain_ms_per_frame": round(ms_p, 3),
        "speedup_vs_plain": round(ms_p / ms_c, 3),
        "rel_mse": mean("rel_mse"), "rel_mse_affected": mean("rel_mse_affected"),
        "truncation_rel_mse": mean("trunc_rel_mse"), "truncation_rel_mse_affected": mean("trunc_rel_mse_affected"),
        "affected_pixel_frac": round(mean("affected"), 4),
        "meets_target": bool(mean("rel_mse") <= 1e-2 and mean("rel_mse_affected") <= 1e-2 and ms_c < ms_p),
        "target": "relative MSE <= 1e-2 over the whole image and over the pixels the depth-2 cut-off changes, "
                  "and a shorter frame than the plain one, after the warm-up frames given",
        "after_32_warmup_frames": None if not early_rows else {
            "warmup_frames": early, "frames": len(early_rows),
            "rel_mse": float(np.mean([r["rel_mse"] for r in early_rows])),
            "rel_mse_affected": float(np.mean([r["rel_mse_affected"] for r in early_rows])),
            "truncation_rel_mse": float(np.mean([r["trunc_rel_mse"] for r in early_rows])),
            "truncation_rel_mse_affected": float(np.mean([r["trunc_rel_mse_affected"] for r in early_rows])),
            "meets_error_target": bool(np.mean([r["rel_mse"] for r in early_rows]) <= 1e-2 and
                                       np.mean([r["rel_mse_affected"] for r in early_rows]) <= 1e-2)},
        "reference": "the plain frame of the same frame number" if ref is None else
                 f"mean of {args.gi_ref_frames} plain path-traced frames (other frame numbers)",
        "plain_rel_mse": None if ref is None else mean("plain_rel_mse"),
        "mrays_per_s": round((mean("rays") + mean("target_rays")) / (ms_c / 1e3) / 1e6, 1),
        "rays_per_frame": int(mean("rays")), "target_rays_per_frame": int(mean("target_rays")),
        "plain_rays_per_frame": int(mean("plain_rays")), "queries_per_frame": int(q),
        "warmup_frames": warm, "frames": n, "train_samples": 65536, "train_steps": 4, "lr": 1e-3,
        "kernel_ms_per_frame": {k: round(v[0] / n, 3) for k, v in kt_c.items()},
        "plain_kernel_ms_per_frame": {k: round(v[0] / n, 3) for k, v in kt_p.items()},
        "mlp_roofline": {"bound": "mfma", "kernel": "k_mlp_forward<1> (inference)",
                         "achieved": round(inf_tflops, 2) if inf_tflops else None,
                         "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(inf_tflops / MFMA_BF16_PEAK_TFLOPS, 4) if inf_tflops else None,
                         "flop_per_query": MLP_FWD_FLOP, "traffic": None,
                         "store_only": {"achieved": round(so_tflops, 2) if so_tflops else None,
                                        "frac": round(so_tflops / MFMA_BF16_PEAK_TFLOPS, 4) if so_tflops else None,
                                        "what": "rt_mlp_forward on as many random feature rows: outputs stored, "
                                                "no per-pixel atomic adds"}},
        "mlp_train": {"achieved": round(tr_tflops, 2) if tr_tflops else None, "unit": "TFLOP/s",
                      "flop_per_sample": MLP_TRAIN_FLOP, "ms_per_frame": round(tr_ms, 3)},
    }
    log(f"cache {ms_c:.2f} ms vs plain {ms_p:.2f} ms ({ms_p / ms_c:.2f}x); rel-MSE {out['rel_mse']:.2e} "
        f"(affected {out['rel_mse_affected']:.2e}); truncation {out['truncation_rel_mse']:.2e} "
        f"(affected {out['truncation_rel_mse_affected']:.2e}); infer {inf_tflops} TFLOP/s (store-only {so_tflops}), "
        f"train {tr_tflops} TFLOP/s")
    return out


def bench_refit(args):
    """Dynamic scene (f4): every icosphere of the c2 scene moves each frame and the BVH is refit on the GPU
    (rt_scene_refit, same tree) instead of rebuilt on the host.  value = refit time per frame (HIP events around
    the refit launches); beside it the host SAH build of the same scene, and the frame time through the refit
    tree against a tree built for the final positions (the refit tree's quality loss)."""
    import numpy as np
    import torch
    from paper_1504_03151_amd import rt, scenes
    w = workload("c2")
    layout = args.layout if args.layout is not None else rt.LAYOUT_BVH4Q
    tile = args.tile or 0
    chunk = args.queue_chunk or 128
    t0 = time.perf_counter()
    sc = rt.Scene(w.scene, node_layout=layout)
    build_s = time.perf_counter() - t0
    sc.upload()
    n_obj = 1000
    tris0 = torch.from_numpy(w.scene.tris.reshape(n_obj, -1, 9)).cuda()
    rng = np.random.default_rng(9)
    vel = torch.from_numpy(rng.uniform(-0.25, 0.25, (n_obj, 1, 3)).astype(np.float32)).cuda()
    frames = max(args.steps, 1) * 4

    def positions(f):
        return (tris0 + (vel * f).repeat(1, 1, 3)).reshape(-1).contiguous()

    for f in range(args.warmup + 1):
        sc.refit(None, positions(f))
    torch.cuda.synchronize()
    ms = []
    for f in range(1, frames + 1):
        p = positions(f)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        sc.refit(None, p)
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    refit_ms = float(np.median(ms))
    # frames through the refit tree vs a tree built for the final positions
    final = positions(frames).cpu().numpy().reshape(-1, 3, 3)
    moved = scenes.make_scene(tris=final, tri_mat=w.scene.tri_mat, materials=w.scene.materials,
                              lights=w.scene.lights)

    def frame_ms(scene):
        r = rt.Renderer(scene, w.camera, w.params, queue_chunk=chunk, tile=tile)
        r.render(rt.FLAG_COUNT_WORK | rt.FLAG_SYNC | rt.FLAG_NO_GRAPH)
        st = r.read_stats()
        for _ in range(2):
            r.render()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            r.render()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / args.steps, st["node_visits"] + st["shadow_node_visits"]

    refit_frame_ms, refit_visits = frame_ms(sc)
    t0 = time.perf_counter()
    sm = rt.Scene(moved, node_layout=layout)
    rebuild_s = time.perf_counter() - t0
    sm.upload()
    fresh_frame_ms, fresh_visits = frame_ms(sm)
    # algorithmic bytes of one refit: positions read (36 B per triangle), primitive records read and written
    # (2 x 48 B) and normals written (16 B), each node's box written (node bytes) plus its side box (24 B)
    n_tri = len(w.scene.tris)
    nb = rt.NODE_BYTES[layout]
    algo = n_tri * (36 + 96 + 16) + sc.info["n_nodes"] * (nb + 24) + n_tri * 48
    achieved = algo / (refit_ms / 1e3) / 1e9
    log(f"refit {refit_ms:.3f} ms (host build {build_s:.2f} s); frame through refit tree {refit_frame_ms:.2f} ms "
        f"vs rebuilt {fresh_frame_ms:.2f} ms; node visits {refit_visits} vs {fresh_visits}")
    # the batch of 256 uneven scenes, every primitive moving: all scenes refit on one stream vs the host build
    ws = scenes.config3(256)
    t0 = time.perf_counter()
    scs = build_scenes(ws, rt)
    batch_build_s = time.perf_counter() - t0
    for x in scs:
        x.upload()
    moved_pos = []
    for b, wb in enumerate(ws):
        g = np.random.default_rng(100 + b)
        sp = wb.scene.spheres.copy()
        if len(sp):
            sp[:, :3] += g.uniform(-0.3, 0.3, (len(sp), 3)).astype(np.float32)
        tr = (wb.scene.tris + g.uniform(-0.3, 0.3, (len(wb.scene.tris), 1, 3))).astype(np.float32)
        moved_pos.append((torch.from_numpy(sp).cuda() if len(sp) else None,
                          torch.from_numpy(np.ascontiguousarray(tr)).cuda() if len(tr) else None))
    for x, (sp, tr) in zip(scs, moved_pos):   # warm-up (workspaces allocated)
        x.refit(sp, tr)
    torch.cuda.synchronize()
    a, bev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for x, (sp, tr) in zip(scs, moved_pos):
        x.refit(sp, tr)
    bev.record()
    torch.cuda.synchronize()
    batch_refit_ms = a.elapsed_time(bev)
    br = rt.BatchRenderer(scs, [wb.camera for wb in ws], [wb.params for wb in ws])
    br.render(rt.FLAG_SYNC)
    assert br.read_stats()["status"] == 0
    log(f"c3 batch: refit of 256 scenes {batch_refit_ms:.2f} ms vs host build {batch_build_s:.2f} s")
    out = {
        "metric": "ms per BVH refit on the GPU (c2 scene, 1.28M triangles, every object moving)",
        "value": round(refit_ms, 4), "unit": "ms", "n_gpus": 1, "steps": frames, "warmup": args.warmup + 1,
        "ms_per_step": round(refit_ms, 4), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c2_icospheres_moving", "triangles": n_tri, "node_layout": layout,
                   "nodes": sc.info["n_nodes"], "frames": frames},
        "host_build_seconds": round(build_s, 3), "host_rebuild_seconds": round(rebuild_s, 3),
        "speedup_vs_host_build": round(build_s * 1e3 / refit_ms, 1),
        "frame_ms_refit_tree": round(refit_frame_ms, 3), "frame_ms_rebuilt_tree": round(fresh_frame_ms, 3),
        "c3_batch_refit_ms": round(batch_refit_ms, 3), "c3_batch_host_build_seconds": round(batch_build_s, 3),
        "c3_batch_triangles": int(sum(len(wb.scene.tris) for wb in ws)),
        "node_visits_refit_tree": int(refit_visits), "node_visits_rebuilt_tree": int(fresh_visits),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "refit (all launches)",
                     "bytes_per_refit": int(algo)},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", help="c0, c1, c2 (default), c3 (the batch) or gi (diffuse global "
                                                         "illumination in a closed room, depth 6)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--graph", action="store_true", help="time graph replays (no per-kernel events)")
    ap.add_argument("--samples-per-pass", type=int, default=0, help="0 = chosen by the library")
    ap.add_argument("--queue-chunk", type=int, default=0, help="0 = library default")
    ap.add_argument("--n-scenes", type=int, default=256, help="scenes of the c3 batch")
    ap.add_argument("--no-cache", action="store_true", help="skip the learned-form comparison")
    ap.add_argument("--progressive", action="store_true",
                    help="progressive passes with disk lights (radius --area-lights, default 2) instead of frames")
    ap.add_argument("--refit", action="store_true",
                    help="dynamic c2 scene: GPU BVH refit per frame vs the host build")
    ap.add_argument("--area-lights", type=float, default=0.0, metavar="R",
                    help="replace the point lights by disks of radius R facing the scene centre (sampled once per "
                         "light per pass)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the given (or default) tile, queue chunk and node layout instead of tuning them")
    ap.add_argument("--tile", type=int, default=None, help="primary-ray tile (0 8x8, 1 16x4, 2 32x2, 3 4x16); "
                                                           "with --layout and --queue-chunk: no tuning")
    ap.add_argument("--layout", type=int, default=None, help="BVH node layout (0 depth-first, 1 breadth-first, "
                                                             "2 treelets)")
    ap.add_argument("--cache-warmup", type=int, default=None,
                    help="online-training frames before measuring (default 256, ~3 s of frames; 96 for "
                         "path-traced frames)")
    ap.add_argument("--cache-frames", type=int, default=16, help="measured learned-form frames")
    ap.add_argument("--gi-ref-frames", type=int, default=8,
                    help="plain path-traced frames averaged into the reference of the learned form (workload gi)")
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
              f"pixels or sample passes across GPUs and sum the accumulators", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1504_03151_amd import rt
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    rt.lib()
    if args.workload == "c3":
        return bench_batch(args)
    if args.progressive:
        return bench_progressive(args)
    if args.refit:
        return bench_refit(args)
    w = workload(args.workload, args.area_lights)
    log(f"workload {w.name}: {len(w.scene.spheres)} spheres, {len(w.scene.tris)} triangles, "
        f"{len(w.scene.planes)} planes, {len(w.scene.lights)} lights")
    t0 = time.perf_counter()
    sc = rt.Scene(w.scene)
    log(f"BVH build {time.perf_counter() - t0:.2f} s: {sc.info}")
    sc.upload()
    chunk, tile, tuned = args.queue_chunk, args.tile or 0, None
    if args.layout:
        sc.set_layout(args.layout).upload()
    if not (args.no_autotune or fixed_config(args)):
        from paper_1504_03151_amd import autotune
        t0 = time.perf_counter()
        tuned = autotune.tune([sc], [w.camera], [w.params], batch=False, log=log)
        chunk, tile = tuned["config"]["chunk"], tuned["config"]["tile"]
        log(f"autotune {time.perf_counter() - t0:.1f} s: {tuned['config']} {tuned['ms']:.3f} ms "
            f"(defaults {tuned['default_ms']:.3f} ms)")
    r = rt.Renderer(sc, w.camera, w.params, samples_per_pass=args.samples_per_pass, queue_chunk=chunk, tile=tile)
    log(f"workspace {r.ws_bytes / 2 ** 30:.2f} GiB")

    # untimed counting frame: rays per depth and BVH work of every traversal launch
    r.render(rt.FLAG_COUNT_WORK | rt.FLAG_SYNC | rt.FLAG_NO_GRAPH)
    cst = r.read_stats()
    assert cst["status"] == 0, cst
    rays = sum(cst["rays"])
    shadow = sum(cst["shadow"])
    log(f"rays/frame {rays} closest-hit + {shadow} shadow; passes {cst['passes']}; per depth closest "
        f"{cst['rays'][:w.params.max_depth + 1]} shadow {cst['shadow'][:w.params.max_depth + 1]}")

    # Every recorded HIP event leaves the GPU idle for a few microseconds, so the timed frames record events
    # around the launches of the dominant traversal kernel only (found in one untimed frame that times them
    # all); the per-kernel split comes from as many untimed frames afterwards.
    dom = None
    flags = 0
    if not args.graph:
        r.render(rt.FLAG_TIME_KERNELS | rt.FLAG_SYNC)
        k0 = rt.kernel_times(reset=True)
        dom = max(("extend", "shadow"), key=lambda k: k0[k][0])
        flags = rt.FLAG_TIME_SHADOW if dom == "shadow" else rt.FLAG_TIME_KERNELS
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
    kt_timed = rt.kernel_times(reset=True)
    st = r.read_stats()
    assert st["status"] == 0, st
    ms = (t1 - t0) * 1e3 / args.steps
    value = (rays + shadow) / (ms / 1e3) / 1e6
    kt = kt_timed
    if not args.graph:
        for _ in range(args.steps):
            r.render(rt.FLAG_TIME_KERNELS)
        torch.cuda.synchronize()
        kt = rt.kernel_times(reset=True)
    log(f"{ms:.2f} ms/frame, {value:.1f} Mrays/s; kernel ms (separate frames) {kt}")

    roof = None
    if not args.graph:
        nb = rt.NODE_BYTES[sc.info["node_layout"]]      # bytes per node fetch
        per = {
            "extend": nb * cst["node_visits"] + 48 * cst["tri_tests"] + 32 * cst["sphere_tests"],
            "shadow": nb * cst["shadow_node_visits"] + 48 * cst["shadow_tri_tests"] + 32 * cst["shadow_sphere_tests"],
        }
        launches_per_frame = kt_timed[dom][1] / args.steps
        avg_launch_s = kt_timed[dom][0] / 1e3 / kt_timed[dom][1]
        bytes_per_launch = per[dom] / launches_per_frame
        achieved = bytes_per_launch / avg_launch_s / 1e9
        traffic = traffic_record(f"k_{dom}", w.name, tile, sc.info["node_layout"], chunk or 128)
        valu = profile_record("valu-record", f"k_{dom}", w.name, tile, sc.info["node_layout"], chunk or 128)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": f"k_{dom}",
                "achieved_is": "algorithmic bytes (node, triangle and sphere records the BVH traversal fetches, "
                               "counted per launch) / HIP-event launch time",
                "frac_hbm_measured": None if traffic is None else round(traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4),
                "frac_valu": None, "valu": None,
                "avg_launch_ms": round(avg_launch_s * 1e3, 4), "bytes_per_launch": int(bytes_per_launch),
                "avg_launch_is": "HIP events around the kernel's launches inside the timed frames",
                "kernel_ms_per_frame": {k: round(v[0] / args.steps, 3) for k, v in kt.items()},
                "kernel_ms_per_frame_is": "HIP events around every traversal and shading launch, in as many "
                                          "frames again after the timed ones"}
        if valu is not None:
            lane_ops = float(valu["valu_lane_ops_per_launch"])
            roof["frac_valu"] = round(lane_ops / avg_launch_s / VALU_PEAK_LANE_OPS, 4)
            roof["valu"] = {"lane_ops_per_launch": lane_ops, "peak_lane_ops_per_s": VALU_PEAK_LANE_OPS,
                            "issue_frac": round(valu["valu_insts_per_launch"] / avg_launch_s / VALU_PEAK_WAVE_INSTS, 4),
                            "lane_utilisation": valu["lane_utilisation"], "ta_busy": valu.get("ta_busy"),
                            "source": "rocprofv3 SQ counters, profiles/ valu-record"}

    cache = None
    if not args.no_cache and (w.name.startswith("c2") or w.params.gi) and not args.area_lights:
        log(f"learned form (radiance cache below depth 2) vs plain depth {w.params.max_depth}")
        cache = bench_cache(w, sc, r, args)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(w, args.cpu_seconds, scene=sc)

    out = {
        "metric": "Mrays/s (closest-hit + shadow rays per second), " +
                  (f"depth-{w.params.max_depth} path-traced frame with diffuse global illumination" if w.params.gi
                   else f"plain depth-{w.params.max_depth} Whitted frame") +
                  (f", disk lights of radius {args.area_lights:g}" if args.area_lights else ""),
        "value": round(value, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "ms_per_frame": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "width": w.camera.width, "height": w.camera.height, "spp": w.params.spp,
                   "max_depth": w.params.max_depth, "triangles": len(w.scene.tris),
                   "spheres": len(w.scene.spheres), "lights": len(w.scene.lights),
                   "rays_per_frame": rays, "shadow_rays_per_frame": shadow, "parallelism": "single-gpu",
                   "tile": rt.TILE_SHAPES[tile], "queue_chunk": chunk or 128, "node_layout": sc.info["node_layout"]},
        "roofline": roof,
        "autotune": None if tuned is None else {"config": tuned["config"], "ms": tuned["ms"],
                                                 "default_ms": tuned["default_ms"], "trials": len(tuned["trials"])},
        "radiance_cache": cache,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
