"""The C ABI on the CPU: exports, validation and error paths, BVH invariants.

No compute call here touches a GPU: scene building, validation and the host
FP32 traversal of the packed BVH are host code.
"""
import os
import re

import numpy as np
import pytest

import oracle
from paper_1504_03151_amd import rt, scenes as S

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mirt.h")


def test_library_exports_every_declared_symbol():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(rt_[a-z_]+)\s*\(", src))
    assert len(names) >= 15
    L = rt.lib()
    for n in sorted(names):
        assert hasattr(L, n), f"libmirt.so does not export {n}"
    assert names <= set(rt.SIGNATURES), names - set(rt.SIGNATURES)
    assert rt.lib().rt_version().decode().startswith("mirt")


def _bad(scene, match):
    with pytest.raises(rt.RTError, match=match):
        rt.Scene(scene)


def test_build_scene_rejects_invalid_input():
    good = S.config0().scene
    sp = good.spheres.copy()
    sp[2, 3] = 0.0
    _bad(S.make_scene(spheres=sp, sphere_mat=good.sphere_mat, materials=good.materials, lights=good.lights),
         "INVALID_ARG")
    sp = good.spheres.copy()
    sp[1, 0] = np.nan
    _bad(S.make_scene(spheres=sp, sphere_mat=good.sphere_mat, materials=good.materials, lights=good.lights),
         "INVALID_ARG")
    _bad(S.make_scene(spheres=good.spheres, sphere_mat=np.full(8, 99), materials=good.materials,
                      lights=good.lights), "INVALID_ARG")
    tris = np.zeros((1, 3, 3), np.float32)
    tris[0, 1, 2] = np.inf
    _bad(S.make_scene(tris=tris, tri_mat=[0], materials=good.materials, lights=good.lights), "INVALID_ARG")
    _bad(S.make_scene(planes=[[0, 2, 0, 1]], plane_mat=[0], materials=good.materials, lights=good.lights),
         "INVALID_ARG")
    m = good.materials.copy()
    m[0, 9] = 7
    _bad(S.make_scene(spheres=good.spheres, sphere_mat=good.sphere_mat, materials=m, lights=good.lights),
         "INVALID_ARG")
    li = good.lights.copy()
    li[0, 4] = np.nan
    _bad(S.make_scene(spheres=good.spheres, sphere_mat=good.sphere_mat, materials=good.materials, lights=li),
         "INVALID_ARG")


def test_bvh_depth_limit_is_an_error():
    w = S.config0()
    tris = S.icosphere(2).astype(np.float32)
    sc = S.make_scene(tris=tris, tri_mat=np.zeros(len(tris)), materials=w.scene.materials, lights=w.scene.lights)
    with pytest.raises(rt.RTError, match="BVH_DEPTH"):
        rt.Scene(sc, max_depth=2)
    assert rt.Scene(sc).info["depth"] <= 60


def test_identical_triangles_build_and_tie_to_the_smallest_id():
    tri = np.array([[[-1, -1, 5], [1, -1, 5], [0, 1, 5]]], np.float32)
    tris = np.repeat(tri, 100, axis=0)
    w = S.config0()
    sc = S.make_scene(tris=tris, tri_mat=np.zeros(100), materials=w.scene.materials, lights=w.scene.lights)
    s = rt.Scene(sc)
    t, ids = s.host_trace(rt.make_rays([[0, 0, 0]], [[0, 0, 1]]))
    assert ids[0] == 0 and t[0] == 5.0


def test_workspace_and_render_argument_errors():
    w = S.config0()
    s = rt.Scene(w.scene)
    cam = rt.camera_c(w.camera)
    p = rt.params_c(w.params)
    import ctypes as C
    assert rt.lib().rt_render_workspace_bytes(s.handle, C.byref(cam), C.byref(p)) > 0
    cam.width = 0
    assert rt.lib().rt_render_workspace_bytes(s.handle, C.byref(cam), C.byref(p)) == 0
    assert b"width" in rt.lib().rt_last_error()
    cam = rt.camera_c(w.camera)
    # not uploaded: refused before any device work
    st = rt.lib().rt_render(s.handle, C.byref(cam), C.byref(p), 256, None)
    assert st == -7
    p.spp = 0
    assert rt.lib().rt_render_workspace_bytes(s.handle, C.byref(cam), C.byref(p)) == 0


@pytest.mark.parametrize("layout", [rt.LAYOUT_DFS, rt.LAYOUT_BVH4, rt.LAYOUT_BVH4Q])
def test_host_traversal_matches_brute_force_on_tiny_scenes(layout):
    for seed in range(6):
        w = S.random_tiny(seed, n_spheres=6, n_tris=80)
        s = rt.Scene(w.scene, node_layout=layout)
        rng = np.random.default_rng(100 + seed)
        o = rng.uniform(-6, 6, (3000, 3))
        d = rng.normal(size=(3000, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        R = rt.make_rays(o, d)
        t, ids, work = s.host_trace(R, with_work=True)
        o32, d32 = R[:, :3].astype(np.float64), R[:, 3:6].astype(np.float64)
        tr, ir, m = oracle.closest(w.scene, o32, d32)
        rob = m > oracle.ROBUST
        assert rob.mean() > 0.98
        assert (ids[rob] == ir[rob]).all()
        assert (work[:, 0] >= 1).all()                       # the root is always fetched
        tm = rng.uniform(0.5, 9, 3000).astype(np.float32)
        R2 = rt.make_rays(o, d, tm)
        _, oid = s.host_trace(R2, any_hit=True)
        occ, m2 = oracle.occluded(w.scene, o32, d32, R2[:, 7].astype(np.float64))
        rob = m2 > oracle.ROBUST
        assert ((oid >= 0)[rob] == occ[rob]).all()


def test_bvh_info_and_work_counts_are_sane():
    w = S.config1(width=64, height=36, grid=128)
    s = rt.Scene(w.scene)
    info = s.info
    assert info["n_bvh_prims"] == len(w.scene.tris) + len(w.scene.spheres)
    assert info["n_leaves"] == info["n_nodes"] + 1             # binary tree: leaves = inner nodes + 1
    assert info["stack_size"] == info["depth"] + 3
    lo, hi = np.array(info["bounds_lo"]), np.array(info["bounds_hi"])
    assert (lo <= w.scene.tris.reshape(-1, 3).min(0)).all() and (hi >= w.scene.tris.reshape(-1, 3).max(0)).all()
    o, d = oracle.camera_rays(w.camera, w.params, np.arange(64 * 36))
    t, ids, work = s.host_trace(rt.make_rays(o, d), with_work=True)
    # a BVH visits far fewer primitives than brute force
    assert work[:, 1].mean() < 0.01 * len(w.scene.tris)


@pytest.mark.parametrize("layout", [rt.LAYOUT_BFS, rt.LAYOUT_TREELET, rt.LAYOUT_BVH4, rt.LAYOUT_BVH4Q])
def test_node_layouts_keep_every_hit_and_every_traversal_step(layout):
    """A node layout only renumbers nodes: the same rays must see the same hits (bit-equal t and id) and fetch
    the same number of nodes and primitives as in depth-first order, for closest and any hit.  The four-wide
    collapse of the same tree must give the same closest hits (bit-equal) and the same any-hit answers, with
    fewer node fetches."""
    w = S.config1(width=64, height=36, grid=96)
    base = rt.Scene(w.scene)
    other = rt.Scene(w.scene, node_layout=layout)
    assert other.info["node_layout"] == layout and base.info["node_layout"] == rt.LAYOUT_DFS
    wide = layout in (rt.LAYOUT_BVH4, rt.LAYOUT_BVH4Q)
    if wide:
        assert other.info["n_nodes"] < 0.6 * base.info["n_nodes"]
    else:
        assert other.info["n_nodes"] == base.info["n_nodes"] and other.info["depth"] == base.info["depth"]
    rng = np.random.default_rng(7)
    o = rng.uniform(-100, 100, (4000, 3)) * [1, 0, 1] + [0, 40, 0]
    d = rng.normal(size=(4000, 3)) - [0, 1.5, 0]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    for any_hit in (False, True):
        R = rt.make_rays(o, d, 150.0 if any_hit else None)
        t0, i0, w0 = base.host_trace(R, any_hit=any_hit, with_work=True)
        t1, i1, w1 = other.host_trace(R, any_hit=any_hit, with_work=True)
        assert (i0 >= 0).mean() > 0.3
        if any_hit and wide:                  # any hit: the same answer, possibly another blocker
            np.testing.assert_array_equal(i0 >= 0, i1 >= 0)
            continue
        np.testing.assert_array_equal(i0, i1)
        np.testing.assert_array_equal(t0, t1)
        if wide:
            assert w1[:, 0].sum() < 0.75 * w0[:, 0].sum()
        else:
            np.testing.assert_array_equal(w0, w1)
    # re-layout of a built scene, and back: identical again; the device copy is dropped
    other.set_layout(rt.LAYOUT_DFS)
    assert other.info["node_layout"] == rt.LAYOUT_DFS and other.blob is None
    R = rt.make_rays(o, d)
    np.testing.assert_array_equal(base.host_trace(R)[1], other.host_trace(R)[1])
    with pytest.raises(rt.RTError, match="INVALID_ARG"):
        other.set_layout(5)
    with pytest.raises(rt.RTError, match="INVALID_ARG"):
        rt.Scene(w.scene, node_layout=-1)


def test_tile_shapes_are_validated_and_size_the_workspace():
    import ctypes as C
    w = S.config0()
    s = rt.Scene(w.scene)
    cam = rt.camera_c(w.camera)
    sizes = []
    for tile in (rt.TILE_8X8, rt.TILE_16X4, rt.TILE_32X2, rt.TILE_4X16):
        p = rt.params_c(w.params, tile=tile)
        sizes.append(rt.lib().rt_render_workspace_bytes(s.handle, C.byref(cam), C.byref(p)))
    assert all(n > 0 for n in sizes)
    p = rt.params_c(w.params, tile=4)
    assert rt.lib().rt_render_workspace_bytes(s.handle, C.byref(cam), C.byref(p)) == 0
    assert b"tile" in rt.lib().rt_last_error()


def test_area_light_records_are_validated():
    good = S.config0().scene
    li = np.zeros((1, 13), np.float32)
    li[0, :6] = [0, 5, 0, 1, 1, 1]
    li[0, 6] = 7                                   # unknown shape
    _bad(S.make_scene(spheres=good.spheres, sphere_mat=good.sphere_mat, materials=good.materials, lights=li),
         "INVALID_ARG")
    li[0, 6] = S.DISK
    li[0, 7:10] = [np.inf, 0, 0]
    _bad(S.make_scene(spheres=good.spheres, sphere_mat=good.sphere_mat, materials=good.materials, lights=li),
         "INVALID_ARG")
    li[0, 7:10] = [1, 0, 0]
    li[0, 10:13] = [0, 0, 1]
    rt.Scene(S.make_scene(spheres=good.spheres, sphere_mat=good.sphere_mat, materials=good.materials, lights=li))


def test_refit_argument_errors_need_no_gpu():
    """rt_scene_refit checks its arguments on the host before any device work."""
    w = S.random_tiny(1, n_spheres=3, n_tris=20, size=8)
    sc = rt.Scene(w.scene)
    L = rt.lib()
    need = L.rt_scene_refit_workspace_bytes(sc.handle)
    assert need >= 24 * sc.info["n_nodes"]
    # not uploaded
    assert L.rt_scene_refit(sc.handle, None, None, None, 0, 0, None) == -7      # RT_ERR_NOT_UPLOADED
    assert L.rt_scene_refit(None, None, None, None, 0, 0, None) == -1           # RT_ERR_INVALID_ARG
    assert b"NULL scene" in L.rt_last_error()
    # the refit order is part of the blob: one int32 per node after the lights
    assert sc.device_bytes >= 4 * sc.info["n_nodes"]


def test_autotune_signature_separates_path_tracing():
    from paper_1504_03151_amd import autotune
    w = S.random_tiny(1, size=8)

    class _S:   # the signature only reads the source arrays
        src = w.scene
    a = autotune.signature([_S()], [w.camera], [w.params])
    w.params.gi = 1
    assert autotune.signature([_S()], [w.camera], [w.params]) != a


def test_global_illumination_room_is_closed():
    """Every camera ray of the path-traced room workload hits something (the walls close it)."""
    import oracle
    w = S.config_gi(width=64, height=36, spp=1)
    o, d = oracle.camera_rays(w.camera, w.params, np.arange(w.camera.n_pixels))
    t, ids, _ = oracle.closest(w.scene, o, d)
    assert (ids >= 0).all()
    assert w.params.gi == 1 and w.params.max_depth == 6


def test_network_entry_points_reject_unaligned_operands_without_a_gpu():
    """rt_mlp_forward / rt_mlp_grad read weights and features as 16-byte vectors: misaligned pointers are
    argument errors, caught on the host before any device work."""
    L = rt.lib()
    for w, x in ((0x1002, 0x2000), (0x1000, 0x2008)):
        assert L.rt_mlp_forward(w, x, 5, 0x3000, None) == -1
        assert b"16-byte aligned" in L.rt_last_error()
        assert L.rt_mlp_grad(w, x, 0x3000, 5, 5, 0x4000, 0x5000, None) == -1
        assert b"16-byte aligned" in L.rt_last_error()
    assert L.rt_mlp_forward(0x1000, 0x2000, 0, 0x3000, None) == 0      # nothing to do


def test_autotune_cache_survives_corrupt_files(tmp_path):
    """A corrupt or malformed autotune cache is never applied: the tuner falls back to tuning from the
    defaults, and writing replaces the file whole."""
    from paper_1504_03151_amd import autotune
    path = str(tmp_path / "tune.json")
    key = "dev|seq|abc"
    good = {"config": {"layout": 4, "chunk": 128, "tile": 0}, "ms": 19.3, "default_ms": 22.8, "trials": []}
    assert autotune.read_cache(path, key) is None                       # missing file
    for junk in ("{not json", "[1, 2, 3]", '{"dev|seq|abc": 5}', "\x00\xff",
                 '{"dev|seq|abc": {"config": {"layout": 9, "chunk": 128, "tile": 0}, "ms": 1.0}}',
                 '{"dev|seq|abc": {"config": {"layout": 4, "chunk": 100, "tile": 0}, "ms": 1.0}}',
                 '{"dev|seq|abc": {"config": {"layout": 4, "chunk": 128}, "ms": 1.0}}'):
        with open(path, "w", errors="surrogateescape") as f:
            f.write(junk)
        msgs = []
        assert autotune.read_cache(path, key, msgs.append) is None, junk
        assert msgs, junk
    autotune.write_cache(path, key, good)                               # replaces the corrupt file
    assert autotune.read_cache(path, key) == good
    autotune.write_cache(path, "other", good)
    assert autotune.read_cache(path, key) == good and autotune.read_cache(path, "other") == good
    assert [p.name for p in tmp_path.iterdir()] == ["tune.json"]       # no temporary left behind


def test_cache_init_and_checkpoint_reject_non_finite_weights_without_a_gpu(tmp_path):
    """rt_cache_init validates the host weights before any device work; a checkpoint with NaN weights,
    a wrong shape or another format is refused before anything is loaded."""
    L = rt.lib()
    n = rt.mlp_num_params()
    w = np.zeros(n, np.float32)
    w[77] = np.nan
    assert L.rt_cache_init(0x100000, 64, w.ctypes.data, None) == -1
    assert b"non-finite" in L.rt_last_error()
    good = dict(format=np.array("mirt-radiance-cache-1"), capacity=np.array(64),
                w_master=np.zeros(n, np.float32), m=np.zeros(n, np.float32), v=np.zeros(n, np.float32),
                steps=np.array(3, np.int64))
    p = str(tmp_path / "ok.npz")
    np.savez(p, **good)
    ck = rt.RadianceCache.read_checkpoint(p)
    assert int(ck["steps"]) == 3
    for k, bad in (("w_master", np.full(n, np.nan, np.float32)), ("m", np.zeros(n - 1, np.float32)),
                   ("v", -np.ones(n, np.float32)), ("format", np.array("something-else"))):
        p = str(tmp_path / f"bad_{k}.npz")
        np.savez(p, **dict(good, **{k: bad}))
        with pytest.raises(ValueError):
            rt.RadianceCache.read_checkpoint(p)
