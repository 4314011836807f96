"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar (fixed before any kernel existed): on every ray whose oracle margin
exceeds 1e-4 the primary hit ids match exactly; on pixels whose whole ray tree
is robust, RGB agrees within 1e-3 absolute; at least 98% of the compared
pixels are robust.  Non-robust pixels must still carry a valid id.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1504_03151_amd import scenes as S

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

pytestmark = pytest.mark.gpu

RGB_TOL = 1e-3
ROBUST = 1e-4


@pytest.fixture(scope="module")
def rt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_03151_amd import rt as _rt
    _rt.lib()
    return _rt


def compare(w, rgb, ids, pixels=None, min_robust=0.98, nthreads=0):
    spp = w.params.spp
    g_rgb = rgb.reshape(-1, 3).double().cpu().numpy()
    g_ids = ids.reshape(-1, spp).cpu().numpy()
    if pixels is None:
        pixels = np.arange(w.camera.n_pixels)
    ref = oracle.render(w.scene, w.camera, w.params, pixels, nthreads=nthreads)
    robust = ref["margin"] > ROBUST
    g_rgb, g_ids = g_rgb[pixels], g_ids[pixels]
    n_prims = w.scene.n_prims
    assert ((g_ids >= -1) & (g_ids < n_prims)).all(), "invalid primitive id"
    assert robust.mean() >= min_robust, f"robust fraction {robust.mean():.4f}"
    bad_ids = np.where(robust[:, None] & (g_ids != ref["ids"]))
    assert len(bad_ids[0]) == 0, (f"{len(bad_ids[0])} robust rays with different ids, e.g. pixel "
                                  f"{pixels[bad_ids[0][0]]}: gpu {g_ids[bad_ids][0]} oracle {ref['ids'][bad_ids][0]}")
    err = np.abs(g_rgb - ref["rgb"]).max(axis=1)
    worst = int(np.argmax(np.where(robust, err, -1)))
    assert err[robust].max() <= RGB_TOL, (f"rgb error {err[robust].max():.3e} at pixel {pixels[worst]}: "
                                          f"gpu {g_rgb[worst]} oracle {ref['rgb'][worst]}")
    return ref, robust, err


def render(rt, w, **kw):
    sc = rt.Scene(w.scene).upload()
    rgb, ids, st = rt.render(sc, w.camera, w.params, **kw)
    torch.cuda.synchronize()
    return sc, rgb, ids, st


# ------------------------------------------------------------------ whole images

def test_config0_full_image(rt):
    w = S.config0()
    _, rgb, ids, st = render(rt, w)
    ref, robust, _ = compare(w, rgb, ids)
    # queue counts per depth equal the oracle's query counts up to non-robust pixels
    o_counts = ref["counts"].sum(axis=0)
    slack = (~robust).sum() * 8
    for k in range(w.params.max_depth + 1):
        assert abs(st["rays"][k] - o_counts[k, 0]) <= slack
        assert abs(st["shadow"][k] - o_counts[k, 1]) <= slack


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_tiny_mixed_scenes_every_pixel(rt, seed):
    # spheres + triangles + plane, Phong / mirror / glass, two lights, ragged 37x29 image
    w = S.random_tiny(seed, size=37, depth=4)
    w.camera.height = 29
    _, rgb, ids, _ = render(rt, w)
    compare(w, rgb, ids, min_robust=0.97)          # oracle: 0.9795 (seed 3) to 1.0


def test_one_sphere_silhouette_and_shadow(rt):
    w = S.one_sphere(center=(0.3, -0.2, 0.5), radius=1.3, plane_y=-3.0, size=48)
    w.params.max_depth = 2
    _, rgb, ids, _ = render(rt, w)
    compare(w, rgb, ids)


def test_jittered_spp_and_graph_replay(rt):
    w = S.random_tiny(5, size=24, depth=3)
    w.params.spp, w.params.jitter, w.params.seed, w.params.frame = 9, 1, 77, 3
    sc = rt.Scene(w.scene).upload()
    r = rt.Renderer(sc, w.camera, w.params, samples_per_pass=2)   # 5 passes, the last one partial
    first = [t.clone() for t in r.render()]
    for _ in range(3):                                               # graph replays give the same frame
        again = r.render()
        torch.cuda.synchronize()
        assert torch.equal(again[1], first[1])
        assert torch.allclose(again[0], first[0], atol=1e-5)
    compare(w, first[0], first[1], min_robust=0.98)       # oracle: 0.9983


def test_pass_splits_give_the_same_frame(rt):
    """Passes of 4 samples sum each pixel's depth-0 background and ambient terms over a block's four waves;
    a partial last pass, passes of 3 samples and per-sample output take the per-ray path.  Every split gives
    the same ids and, up to the order of additions, the same image."""
    w = S.random_tiny(6, size=37, depth=3)                 # ragged tiles: dead lanes in the blocks
    w.camera.height = 29
    w.params.spp, w.params.jitter = 10, 1
    sc = rt.Scene(w.scene).upload()
    out = []
    for spp_pass in (10, 4, 3, 8):
        r = rt.Renderer(sc, w.camera, w.params, samples_per_pass=spp_pass)
        rgb, ids = r.render(rt.FLAG_SYNC)
        torch.cuda.synchronize()
        out.append((rgb.clone(), ids.clone()))
    rs = rt.Renderer(sc, w.camera, w.params, per_sample=True)
    rgb_s, ids_s = rs.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    for rgb, ids in out[1:]:
        assert torch.equal(ids, out[0][1])
        assert torch.allclose(rgb, out[0][0], rtol=1e-5, atol=1e-6)
    assert torch.equal(ids_s, out[0][1])
    assert torch.allclose(rgb_s.mean(dim=2), out[0][0], rtol=1e-5, atol=2e-6)
    compare(w, out[1][0], out[1][1], min_robust=0.965)    # oracle: 0.973 (10 samples per pixel)


def test_rays_missing_the_root_end_at_ray_generation(rt):
    """Without planes, ray generation ends the camera rays that reach none of the root's child boxes (89% of
    them here): their background terms are summed per pixel there and their hit ids set to -1.  Every pass
    split, per-sample output and graph replays give the oracle's frame, and the timing flags change nothing:
    RT_FLAG_TIME_SHADOW records events around the shadow launches only."""
    w = S.random_tiny(7, size=37, depth=3, with_plane=False)   # ragged tiles: dead lanes in the blocks
    w.camera.height = 29
    w.params.spp, w.params.jitter = 10, 1
    sc = rt.Scene(w.scene).upload()
    out = []
    for spp_pass in (10, 4, 3):
        r = rt.Renderer(sc, w.camera, w.params, samples_per_pass=spp_pass)
        rgb, ids = r.render(rt.FLAG_SYNC)
        out.append((rgb.clone(), ids.clone()))
        for flags in (rt.FLAG_TIME_SHADOW, rt.FLAG_TIME_KERNELS, 0, 0):   # eager timed frames, graph replays
            rt.kernel_times(reset=True)
            again = r.render(rt.FLAG_SYNC | flags)
            kt = rt.kernel_times(reset=True)
            assert torch.equal(again[1], ids)
            assert torch.allclose(again[0], rgb, rtol=1e-5, atol=1e-6)
            timed = {k for k, (ms, n) in kt.items() if n > 0}
            assert timed == ({"shadow"} if flags == rt.FLAG_TIME_SHADOW else
                             {"extend", "shade", "shadow"} if flags == rt.FLAG_TIME_KERNELS else set()), (flags, kt)
    rs = rt.Renderer(sc, w.camera, w.params, per_sample=True)
    rgb_s, ids_s = rs.render(rt.FLAG_SYNC)
    for rgb, ids in out[1:]:
        assert torch.equal(ids, out[0][1])
        assert torch.allclose(rgb, out[0][0], rtol=1e-5, atol=1e-6)
    assert torch.equal(ids_s, out[0][1])
    assert torch.allclose(rgb_s.mean(dim=2), out[0][0], rtol=1e-5, atol=2e-6)
    assert (out[0][1] == -1).double().mean() > 0.8
    compare(w, out[2][0], out[2][1], min_robust=0.98)      # oracle: 0.9907


def test_edge_cases(rt):
    # empty scene (only background), a planes-only scene, a 1x1 image, depth 0
    bg = (0.25, 0.5, 0.75)
    empty = S.make_scene(materials=np.stack([S.material()]), lights=[[0, 5, 0, 1, 1, 1]])
    cam = S.Camera((0.0, 0.0, -5.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 45.0, 5, 3)
    w = S.Workload(empty, cam, S.Params(max_depth=2, bg=bg), "empty")
    _, rgb, ids, st = render(rt, w)
    assert (ids.cpu().numpy() == -1).all()
    np.testing.assert_allclose(rgb.cpu().numpy().reshape(-1, 3), np.tile(bg, (15, 1)), rtol=0, atol=0)
    planes = S.make_scene(planes=[[0, 1, 0, -1], [0, 0, -1, -20]], plane_mat=[0, 1],
                          materials=np.stack([S.material(k_r=0.5), S.mirror_material()]),
                          lights=[[0, 5, -3, 1, 1, 1]])
    w = S.Workload(planes, S.Camera((0.0, 0.0, -5.0), (0.0, -0.2, 0.0), (0.0, 1.0, 0.0), 70.0, 17, 11),
                   S.Params(max_depth=3), "planes")
    _, rgb, ids, _ = render(rt, w)
    compare(w, rgb, ids, min_robust=0.9)           # oracle: 0.909 (two planes near grazing incidence)
    w = S.config0()
    w.camera.width = w.camera.height = 1
    _, rgb, ids, _ = render(rt, w)
    compare(w, rgb, ids, min_robust=1.0)
    w = S.config0()
    w.params.max_depth = 0
    _, rgb, ids, _ = render(rt, w)
    compare(w, rgb, ids)


# ------------------------------------------------------------------ single rays through rt_intersect / rt_occluded

def _workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _oracle_rays(w, jobs):
    """Every ray the oracle traces for the given (pixel, sample) pairs (its ray log, in recursion order)."""
    with ThreadPoolExecutor(_workers()) as ex:
        recs = list(ex.map(lambda a: oracle.ray_tree(w.scene, w.camera, w.params, int(a[0]), int(a[1]))[0], jobs))
    return np.concatenate(recs, axis=0)


def _uv_normal(uv):
    """Unit normal of a sphere hit from its (longitude / 2 pi, polar angle / pi) surface coordinates."""
    ph, th = 2 * np.pi * uv[:, 0] - np.pi, np.pi * uv[:, 1]
    return np.stack([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)], axis=1)


def _ray_jobs(cfg):
    """(workload, node layout, (pixel, sample) pairs) of the per-ray comparisons.  c2's rays come from
    pixels whose first camera ray hits an object: 16 jittered samples, up to 8 bounces through mirror
    and glass icospheres, 8 lights per hit."""
    if cfg == "tiny":
        w = S.random_tiny(7, size=40, depth=4)
        return w, 0, [(p, 0) for p in S.pixel_subset(w.camera, 600, 11)]
    if cfg == "c0":
        w = S.config0()
        return w, 0, [(p, 0) for p in S.pixel_subset(w.camera, 600, 11)]
    if cfg == "c1":
        w = S.config1()
        return w, 4, [(p, 0) for p in S.pixel_subset(w.camera, 1024, 12)]
    w = S.config2()
    fx = np.load(os.path.join(GOLDEN, "c2_frame_oracle.npz"))
    hit_px = fx["pixels"][fx["ids"][:, 0] >= 0][:32]
    return w, 4, [(p, s) for p in hit_px for s in range(w.params.spp)]


@pytest.mark.parametrize("cfg", ["tiny", "c0", "c1", "c2"])
def test_intersect_and_occluded_on_oracle_rays(rt, cfg):
    """rt_intersect / rt_occluded (Algorithm 1's object loop and blocker loop) on the oracle's own camera,
    secondary and shadow rays, cast to FP32; c1 and c2 through the quantized four-wide nodes the benchmark
    uses.  Robust rays: equal ids, t within 2e-5, equal blocked flags, surface coordinates as the oracle's.
    At least 98% of the rays must be robust (the oracle measures 99.85% or more on every set here)."""
    w, layout, jobs = _ray_jobs(cfg)
    floor = 0.98
    rec = _oracle_rays(w, jobs)
    sc = rt.Scene(w.scene, node_layout=layout).upload()
    ns, nt = len(w.scene.spheres), len(w.scene.tris)
    for shadow in (False, True):
        sel = rec[rec[:, 0] == 3] if shadow else rec[rec[:, 0] != 3]
        R = rt.make_rays(sel[:, 2:5], sel[:, 5:8], sel[:, 8] if shadow else None)
        o32, d32 = R[:, 0:3].astype(np.float64), R[:, 3:6].astype(np.float64)
        Rd = torch.from_numpy(R).cuda()
        if shadow:
            occ = rt.occluded(sc, Rd).cpu().numpy().astype(bool)
            ref, m = oracle.occluded(w.scene, o32, d32, R[:, 7].astype(np.float64), nthreads=_workers())
            rob = m > ROBUST
            assert rob.mean() >= floor, f"shadow rays: robust fraction {rob.mean():.4f}"
            bad = np.where(rob & (occ != ref))[0]
            assert len(bad) == 0, f"{len(bad)} robust shadow rays differ of {rob.sum()}"
        else:
            t, ids, uv = rt.intersect(sc, Rd, uv=True)
            t, ids, uv = t.cpu().numpy(), ids.cpu().numpy(), uv.cpu().numpy().astype(np.float64)
            tr, ir, m, uvr = oracle.closest(w.scene, o32, d32, nthreads=_workers(), uv=True)
            rob = m > ROBUST
            assert rob.mean() >= floor, f"closest-hit rays: robust fraction {rob.mean():.4f}"
            bad = np.where(rob & (ids != ir))[0]
            assert len(bad) == 0, (f"{len(bad)} robust rays with different ids of {rob.sum()}, e.g. gpu "
                                   f"{ids[bad[0]]} oracle {ir[bad[0]]}")
            hit = rob & (ir >= 0)
            np.testing.assert_allclose(t[hit], tr[hit], rtol=2e-5)
            # triangle barycentrics: FP32 edge functions of coordinates relative to the ray origin, so the
            # error grows with the distance and shrinks with the triangle's projected size (tolerance below)
            tri = hit & (ir >= ns) & (ir < ns + nt)
            if tri.any():
                v = w.scene.tris[ir[tri] - ns].astype(np.float64)
                area2 = np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1)
                cosang = np.abs(np.einsum("ij,ij->i", np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]) /
                                          area2[:, None], d32[tri]))
                span = np.abs(o32[tri]).max(axis=1) + tr[tri]
                edge = np.linalg.norm(v - np.roll(v, 1, axis=1), axis=2).max(axis=1)
                tol = 1e-5 + 64 * 2.0 ** -24 * span * edge / (area2 * np.maximum(cosang, 1e-3))
                err = np.abs(uv[tri] - uvr[tri]).max(axis=1)
                worst = int(np.argmax(err / tol))
                assert (err <= tol).all(), f"barycentrics off by {err[worst]:.2e} (tolerance {tol[worst]:.2e})"
            sph = hit & (ir < ns)
            if sph.any():
                dn = np.linalg.norm(_uv_normal(uv[sph]) - _uv_normal(uvr[sph]), axis=1)
                assert dn.max() <= 1e-3, f"sphere normal from uv off by {dn.max():.2e}"
            miss_or_plane = rob & ((ir < 0) | (ir >= ns + nt))
            assert (uv[miss_or_plane] == 0).all()


@pytest.mark.parametrize("layout", [0, 3, 4])      # binary depth-first, four-wide, quantized four-wide
def test_random_rays_bvh_equals_brute_force(rt, layout):
    for seed in range(3):
        w = S.random_tiny(20 + seed, n_spheres=8, n_tris=200)
        sc = rt.Scene(w.scene, node_layout=layout).upload()
        rng = np.random.default_rng(seed)
        o = rng.uniform(-6, 6, (20000, 3))
        d = rng.normal(size=(20000, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        R = rt.make_rays(o, d)
        t, ids = rt.intersect(sc, torch.from_numpy(R).cuda())
        tr, ir, m = oracle.closest(w.scene, R[:, :3].astype(np.float64), R[:, 3:6].astype(np.float64))
        rob = m > ROBUST
        assert rob.mean() > 0.98
        assert (ids.cpu().numpy()[rob] == ir[rob]).all()
        # and the host traversal of the same BVH agrees with the device
        th, ih = sc.host_trace(R)
        assert (ih[rob] == ir[rob]).all()
        # any hit on segments: the device answer is the oracle's on robust rays
        tm = rng.uniform(0.5, 9, 20000).astype(np.float32)
        R2 = rt.make_rays(o, d, tm)
        occ = rt.occluded(sc, torch.from_numpy(R2).cuda()).cpu().numpy().astype(bool)
        oc, m2 = oracle.occluded(w.scene, R2[:, :3].astype(np.float64), R2[:, 3:6].astype(np.float64),
                                 R2[:, 7].astype(np.float64))
        rob2 = m2 > ROBUST
        assert rob2.mean() > 0.97
        assert (occ[rob2] == oc[rob2]).all()


# ------------------------------------------------------------------ full-size configurations, sampled pixels

@pytest.mark.parametrize("layout", [0, 4])       # binary depth-first; quantized four-wide (the tuned layout)
def test_config1_full_frame_sampled(rt, layout):
    """1080p terrain (522,242 triangles) with 64 mirror spheres, depth 5: 4,096 seeded pixels."""
    w = S.config1()
    sc = rt.Scene(w.scene, node_layout=layout).upload()
    rgb, ids, st = rt.render(sc, w.camera, w.params)
    torch.cuda.synchronize()
    assert st["status"] == 0
    pixels = S.pixel_subset(w.camera, 4096, 21)
    compare(w, rgb, ids, pixels, nthreads=_workers())


def test_config2_full_frame_sampled(rt):
    """1080p x 16 spp, depth 8: compared sample by sample (per-sample accumulation).

    With 16 jittered samples per pixel over small icosphere facets, a pixel is
    rarely robust in all 16 ray trees, so the robust filter is applied per
    sample (each sample's whole tree).  The averaged frame is the mean of the
    per-sample frame; fully robust pixels of it are compared as well.
    """
    w = S.config2()
    sc = rt.Scene(w.scene).upload()
    rs = rt.Renderer(sc, w.camera, w.params, per_sample=True)
    rgb_s, ids = rs.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    st = rs.read_stats()
    assert st["status"] == 0 and st["rays"][8] > 0
    # pixels whose primary ray hits an object (the oracle's own primary pass), plus background pixels
    cand = S.pixel_subset(w.camera, 4000, 22)
    o, d = oracle.camera_rays(w.camera, w.params, cand, sample=0)
    _, ih, _ = oracle.closest(w.scene, o, d)
    pixels = np.sort(np.concatenate([cand[ih >= 0][:24], cand[ih < 0][:8]]))
    ref = oracle.render(w.scene, w.camera, w.params, pixels)
    g_s = rgb_s.reshape(-1, w.params.spp, 3).double().cpu().numpy()[pixels]
    g_ids = ids.reshape(-1, w.params.spp).cpu().numpy()[pixels]
    rob = ref["margin_s"] > ROBUST
    assert rob.mean() >= 0.85, f"per-sample robust fraction {rob.mean():.3f}"
    assert (g_ids[rob] == ref["ids"][rob]).all()
    assert ((g_ids >= -1) & (g_ids < w.scene.n_prims)).all()
    err = np.abs(g_s - ref["rgb_s"]).max(axis=2)
    assert err[rob].max() <= RGB_TOL, err[rob].max()
    # the averaged frame (the benchmarked configuration) is the mean of the samples
    ra = rt.Renderer(sc, w.camera, w.params)
    rgb, ids_a = ra.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    assert torch.equal(ids_a, ids)
    assert torch.allclose(rgb, rgb_s.mean(dim=2), atol=2e-5)
    full = ref["margin"] > ROBUST
    g_avg = rgb.reshape(-1, 3).double().cpu().numpy()[pixels]
    assert full.sum() >= 8
    assert np.abs(g_avg - ref["rgb"]).max(axis=1)[full].max() <= RGB_TOL


def test_config2_benchmarked_setting_against_stored_oracle(rt):
    """The benchmarked frame exactly as bench.py times it after autotuning (quantized four-wide nodes, 8x8
    tiles, queue chunk 128; 1080p x 16 jittered spp, depth 8), against the oracle's brute-force render of
    1,024 seeded pixels (512 with an object under the first sample, 512 others) stored by
    tests/golden/make_oracle_fixtures.py.

    Per sample (each sample's whole ray tree): robust samples have the oracle's primary id and radiance
    within 1e-3.  The oracle certifies 95.0% of these samples robust: all of the background pixels' and
    90.1% of the object pixels' (a sample's tree of up to ~200 rays crosses many small facets of mirror
    and glass icospheres, and one decision within the 1e-4 margin anywhere in it excludes the sample).
    That fraction is a property of the scene and the oracle alone; the floor only guards against a
    shrunken comparison set.  The averaged frame is compared on the 718 pixels (70%) all of whose 16
    samples are robust."""
    import sys
    sys.path.insert(0, GOLDEN)
    from make_oracle_fixtures import scene_digest
    fx = np.load(os.path.join(GOLDEN, "c2_frame_oracle.npz"))
    w = S.config2()
    assert str(fx["digest"]) == scene_digest(w), "stored oracle results are for another scene"
    pixels = fx["pixels"]
    sc = rt.Scene(w.scene, node_layout=rt.LAYOUT_BVH4Q).upload()
    rs = rt.Renderer(sc, w.camera, w.params, per_sample=True, tile=0, queue_chunk=128)
    rgb_s, ids = rs.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    st = rs.read_stats()
    assert st["status"] == 0 and st["rays"][8] > 0
    g_s = rgb_s.reshape(-1, w.params.spp, 3).double().cpu().numpy()[pixels]
    g_ids = ids.reshape(-1, w.params.spp).cpu().numpy()[pixels]
    assert ((g_ids >= -1) & (g_ids < w.scene.n_prims)).all()
    rob = fx["margin_s"] > ROBUST
    assert rob.mean() >= 0.94, f"per-sample robust fraction {rob.mean():.4f}"
    bad = np.where(rob & (g_ids != fx["ids"]))
    assert len(bad[0]) == 0, f"{len(bad[0])} robust samples with different primary ids"
    err = np.abs(g_s - fx["rgb_s"]).max(axis=2)
    assert err[rob].max() <= RGB_TOL, f"per-sample rgb error {err[rob].max():.3e}"
    # the averaged frame: the benchmarked output
    ra = rt.Renderer(sc, w.camera, w.params, tile=0, queue_chunk=128)
    rgb, ids_a = ra.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    assert torch.equal(ids_a, ids)
    assert torch.allclose(rgb, rgb_s.mean(dim=2), atol=2e-5)
    full = fx["margin"] > ROBUST
    assert full.sum() >= 700, full.sum()
    g_avg = rgb.reshape(-1, 3).double().cpu().numpy()[pixels]
    assert np.abs(g_avg - fx["rgb"]).max(axis=1)[full].max() <= RGB_TOL


def test_deferred_shadow_queue_capacity(rt):
    """Inside a closed box of reflective Phong walls every ray hits and every hit sends one shadow ray, so the
    deferred shadow queue of a depth-4 frame holds 5 x the primary rays: queue_factor 1 must report the
    overflow (RT_ERR_CAPACITY under FLAG_SYNC), queue_factor 5 must fit exactly and match the oracle."""
    planes = [[1, 0, 0, -5], [-1, 0, 0, -5], [0, 1, 0, -5], [0, -1, 0, -5], [0, 0, 1, -5], [0, 0, -1, -5]]
    scene = S.make_scene(planes=planes, plane_mat=[0] * 6, materials=np.stack([S.material((0.6, 0.5, 0.4), k_r=0.5)]),
                         lights=[[1.0, 2.0, 0.5, 1.0, 1.0, 1.0]], name="mirror_box")
    cam = S.Camera((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0), 60.0, 32, 32)
    p = S.Params(spp=1, max_depth=4, jitter=0, seed=1)
    sc = rt.Scene(scene).upload()
    with pytest.raises(rt.RTError, match="CAPACITY"):
        rt.render(sc, cam, p, queue_factor=1.0)
    rgb, ids, st = rt.render(sc, cam, p, queue_factor=5.0)
    torch.cuda.synchronize()
    assert st["status"] == 0
    assert st["rays"][:5] == [1024] * 5 and st["shadow"][:5] == [1024] * 5
    ref = oracle.render(scene, cam, p)
    rob = ref["margin"] > ROBUST
    assert rob.mean() > 0.94                               # oracle: 0.949 (the box's edges and corners)
    np.testing.assert_allclose(rgb.reshape(-1, 3).cpu().numpy()[rob], ref["rgb"][rob], rtol=0, atol=1e-3)
    assert (ids.reshape(-1).cpu().numpy()[rob] == ref["ids"][rob, 0]).all()
