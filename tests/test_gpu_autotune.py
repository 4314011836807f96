"""Tile shapes, node layouts and the autotuner on the GPU.

Every tile shape and node layout must give the same primary-hit ids as the
default (8x8 tiles, depth-first nodes) and the same image up to the order of
floating-point accumulation; the tuner must return a setting from its space
whose ids it verified, leave the scenes in that layout, and reuse its cache.
"""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1504_03151_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_03151_amd import rt as _rt
    _rt.lib()
    return _rt


def _ragged():
    w = S.random_tiny(4, n_spheres=6, n_tris=60, size=45, depth=4)
    w.camera.height = 29                          # ragged in every tile shape
    w.params.spp, w.params.jitter = 4, 1
    return w


def test_every_tile_and_layout_gives_the_default_frame(rt):
    w = _ragged()
    sc = rt.Scene(w.scene).upload()
    rgb0, ids0, st0 = rt.render(sc, w.camera, w.params)
    rgb0, ids0 = rgb0.clone(), ids0.clone()
    torch.cuda.synchronize()
    for layout in (rt.LAYOUT_DFS, rt.LAYOUT_BFS, rt.LAYOUT_TREELET, rt.LAYOUT_BVH4, rt.LAYOUT_BVH4Q):
        s = rt.Scene(w.scene, node_layout=layout).upload()
        for tile in rt.TILE_SHAPES:
            rgb, ids, st = rt.render(s, w.camera, w.params, tile=tile, queue_chunk=64 if tile % 2 else 256)
            torch.cuda.synchronize()
            assert st["rays"] == st0["rays"] and st["shadow"] == st0["shadow"], (layout, tile)
            assert torch.equal(ids, ids0), (layout, tile)
            assert torch.allclose(rgb, rgb0, rtol=1e-5, atol=1e-6), (layout, tile, (rgb - rgb0).abs().max().item())
    # and the default frame is the oracle's on robust pixels
    ref = oracle.render(w.scene, w.camera, w.params)
    rob = ref["margin"] > 1e-4
    assert rob.mean() > 0.955                              # oracle: 0.9609 (4 jittered samples per pixel)
    assert (ids0.reshape(-1, 4).cpu().numpy()[rob] == ref["ids"][rob]).all()


def test_batched_tiles_per_scene(rt):
    ws = [S.random_tiny(s, size=21 + 5 * s, depth=3) for s in range(4)]
    scs = [rt.Scene(w.scene).upload() for w in ws]
    a = rt.BatchRenderer(scs, [w.camera for w in ws], [w.params for w in ws])
    b = rt.BatchRenderer(scs, [w.camera for w in ws], [w.params for w in ws], tile=[0, 1, 2, 3], queue_chunk=512)
    ra, ia = a.render(rt.FLAG_SYNC)
    rb, ib = b.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    for x, y, u, v in zip(ra, rb, ia, ib):
        assert torch.equal(u, v)
        assert torch.allclose(x, y, rtol=1e-5, atol=1e-6)


def test_autotuner_picks_a_verified_setting_and_caches_it(rt, tmp_path):
    from paper_1504_03151_amd import autotune
    ws = [S.config3_scene(b) for b in range(6)]
    for w in ws:                                  # keep the test short: small images
        w.camera.width = min(w.camera.width, 96)
        w.camera.height = min(w.camera.height, 80)
    scs = [rt.Scene(w.scene).upload() for w in ws]
    cams, ps = [w.camera for w in ws], [w.params for w in ws]
    path = str(tmp_path / "tune.json")
    space = {"layout": autotune.SPACE["layout"], "chunk": [64, 128, 512], "tile": autotune.SPACE["tile"]}
    res = autotune.tune(scs, cams, ps, batch=True, steps=2, rounds=1, space=space, cache_path=path)
    cfg = res["config"]
    assert cfg["layout"] in space["layout"] and cfg["chunk"] in space["chunk"] and cfg["tile"] in space["tile"]
    assert all(t["ids_match"] for t in res["trials"])
    assert len(res["trials"]) >= 5 + 2 + 3
    assert res["ms"] <= res["default_ms"]
    assert all(s.info["node_layout"] == cfg["layout"] and s.blob is not None for s in scs)
    db = json.load(open(path))
    assert res["key"] in db
    again = autotune.tune(scs, cams, ps, batch=True, cache_path=path)
    assert again["cached"] and again["config"] == cfg
    # the tuned setting renders the same ids as the default one
    ref = rt.BatchRenderer(scs, cams, ps)
    tuned = rt.BatchRenderer(scs, cams, ps, queue_chunk=cfg["chunk"], tile=cfg["tile"])
    _, ia = ref.render(rt.FLAG_SYNC)
    _, ib = tuned.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    assert all(torch.equal(u, v) for u, v in zip(ia, ib))
