"""Learned form (radiance cache below depth 2) against the oracle.

* Inference: with fixed weights, the GPU frame equals the oracle's cut-off
  render plus w * max(network(features), 0) of each of its depth-2 hits (the
  network evaluated by oracle/mlp.py), on robust pixels.
* Targets: each training sample's target equals the oracle's radiance of the
  oracle's own depth-2 ray of the same pixel (matched by direction).
* Training frames lower the loss; graph replays reproduce eager frames.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import mlp as M
from paper_1504_03151_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_03151_amd import rt as _rt
    _rt.lib()
    return _rt


def _scene():
    w = S.random_tiny(11, size=40, depth=4)     # spheres, triangles, plane, mirrors and glass
    w.camera.height = 37
    return w


def test_cache_inference_matches_oracle(rt):
    w = _scene()
    sc = rt.Scene(w.scene).upload()
    bounds = (np.array(sc.info["bounds_lo"]) - 1.0, np.array(sc.info["bounds_hi"]) + 1.0)
    ws = S.mlp_init_weights(7)
    ws[5] = np.abs(ws[5])                               # positive outputs: the cache terms are visible
    cache = rt.RadianceCache(ws, capacity=4096)
    r = rt.CachedRenderer(sc, w.camera, w.params, cache, mode=rt.CACHE_INFER, depth=2, bounds=bounds)
    rgb, ids = r.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    assert r.read_stats()["status"] == 0
    ref = oracle.render_cache(w.scene, w.camera, w.params, 2)
    rec = ref["records"]
    assert len(rec) > 50
    feats = M.encode(rec[:, 1:4], rec[:, 4:7], rec[:, 7:10], bounds[0].astype(np.float32),
                     bounds[1].astype(np.float32))
    y, _ = M.forward(ws, feats)
    term = rec[:, 10:13] * np.maximum(y, 0.0)
    img = ref["rgb"].copy()
    cache_mag = np.zeros_like(img)
    np.add.at(img, rec[:, 0].astype(int), term)
    np.add.at(cache_mag, rec[:, 0].astype(int), np.abs(term))
    rob = ref["margin"] > 1e-4
    assert rob.mean() > 0.98                               # oracle: 0.9986
    g = rgb.reshape(-1, 3).double().cpu().numpy()
    err = np.abs(g - img)
    tol = 1e-3 + 3e-2 * cache_mag
    assert (err[rob] <= tol[rob]).all(), (err - tol)[rob].max()
    assert (cache_mag[rob] > 1e-3).sum() > 30                      # the cache really contributes
    # the oracle's ids are the ones of the plain frame (primary rays are unaffected)
    full = oracle.render(w.scene, w.camera, w.params)
    assert (ids.reshape(-1).cpu().numpy()[rob] == full["ids"][rob, 0]).all()


def test_training_targets_match_oracle_radiance(rt):
    w = _scene()
    sc = rt.Scene(w.scene).upload()
    cache = rt.RadianceCache(S.mlp_init_weights(3), capacity=2048)
    r = rt.CachedRenderer(sc, w.camera, w.params, cache, mode=rt.CACHE_TRAIN, depth=2, full_depth=6,
                          train_samples=2048, train_steps=2)
    r.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    c = cache.counters()
    assert c["steps"] == 2 and c["n_train"] > 50
    rays, feats, targets, pix = [t.cpu().numpy() for t in cache.training_batch()]
    p6 = S.Params(spp=1, max_depth=6, jitter=0, seed=w.params.seed, bg=w.params.bg, eps=w.params.eps)
    checked = 0
    for j in range(0, len(rays), max(1, len(rays) // 120)):
        tree, _ = oracle.ray_tree(w.scene, w.camera, w.params, int(pix[j]))
        cand = tree[((tree[:, 0] == 1) | (tree[:, 0] == 2)) & (tree[:, 1] == 2)]
        if not len(cand) or (tree[:, 11] <= 1e-4).any():
            continue
        k = int(np.argmax(cand[:, 5:8] @ rays[j, 3:6]))
        if cand[k, 5:8] @ rays[j, 3:6] < 1 - 1e-6:
            continue
        L, m = oracle.radiance(w.scene, p6, cand[k, 2:5], cand[k, 5:8], 2, so=cand[k, 2:5].max() * 4e-7, sd=4e-7)
        if m[0] <= 1e-4:
            continue
        np.testing.assert_allclose(targets[j], L[0], atol=1e-3, rtol=0)
        checked += 1
    assert checked >= 20, checked


def test_training_frames_lower_the_loss_and_graph_replays_match(rt):
    w = _scene()
    sc = rt.Scene(w.scene).upload()
    cache = rt.RadianceCache(S.mlp_init_weights(5), capacity=2048)
    r = rt.CachedRenderer(sc, w.camera, w.params, cache, mode=rt.CACHE_TRAIN, depth=2, full_depth=6,
                          train_samples=2048, train_steps=4, lr=3e-3)
    losses = []
    for f in range(40):
        w.params.frame = f
        r.render()
        torch.cuda.synchronize()
        c = cache.counters()
        losses.append(float(c["loss_sums"][:4].sum()) / (3 * c["n_train"]))
    assert np.mean(losses[-5:]) < 0.5 * np.mean(losses[:3]), losses
    # inference frames: graph replay == eager frame, same weights
    r.set_mode(rt.CACHE_INFER)
    a = [t.clone() for t in r.render(rt.FLAG_SYNC)]
    r.graph = False
    b = r.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    assert torch.equal(a[1], b[1]) and torch.allclose(a[0], b[0], atol=1e-5)


def test_trained_network_beats_depth2_truncation(rt):
    """What the network gains: after online training, the learned-form image is closer (relative MSE) to the
    oracle's full-depth image than the same frame cut off at depth 2 without the network (parity unpinned:
    training is order- and rounding-dependent, so only this gain is asserted)."""
    w = S.random_tiny(7, size=64, depth=4)          # 176 pixels change when the recursion is cut at depth 2
    sc = rt.Scene(w.scene).upload()
    cache = rt.RadianceCache(S.mlp_init_weights(9), capacity=2048)
    r = rt.CachedRenderer(sc, w.camera, w.params, cache, mode=rt.CACHE_TRAIN, depth=2,
                          full_depth=w.params.max_depth, train_samples=2048, train_steps=4, lr=3e-3)
    for f in range(80):
        w.params.frame = f
        r.render()
    r.set_mode(rt.CACHE_INFER)
    rgb, _ = r.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    img = rgb.reshape(-1, 3).double().cpu().numpy()
    full = oracle.render(w.scene, w.camera, w.params)["rgb"]
    trunc = oracle.render_cache(w.scene, w.camera, w.params, 2)["rgb"]
    aff = (np.abs(full - trunc) > 1e-6).any(axis=1)
    assert aff.sum() > 150, aff.sum()
    e_net = M.rel_mse(img[aff], full[aff])
    e_cut = M.rel_mse(trunc[aff], full[aff])
    print(f"affected pixels {aff.sum()}: rel-MSE network {e_net:.3e}, truncation {e_cut:.3e}")
    assert e_net < 0.5 * e_cut, (e_net, e_cut)
    assert M.rel_mse(img, full) < M.rel_mse(trunc, full)


def test_learned_form_full_frame_sampled(rt):
    """c4 at full size (1080p x 16 spp, 1.28M triangles, ~1M network queries per frame, the benchmarked
    launch configuration), fixed weights: sampled pixels, most of them reached by the cache terms (found
    as the difference to the same frame with a zero network), against the oracle's cut-off render plus
    w * max(network(features), 0) / spp of its depth-2 hits, on pixels robust in all 16 ray trees."""
    w = S.config2()
    spp = w.params.spp
    sc = rt.Scene(w.scene).upload()
    bounds = (np.array(sc.info["bounds_lo"], np.float32), np.array(sc.info["bounds_hi"], np.float32))
    ws = S.mlp_init_weights(7)
    ws[5] = np.abs(ws[5])                               # positive outputs: the cache terms are visible
    frames = []
    for weights in (ws, [np.zeros_like(x) for x in ws]):
        cache = rt.RadianceCache(weights, capacity=4096)
        r = rt.CachedRenderer(sc, w.camera, w.params, cache, mode=rt.CACHE_INFER, depth=2, full_depth=8,
                              bounds=bounds, with_ids=False)
        rgb, _ = r.render(rt.FLAG_SYNC)
        torch.cuda.synchronize()
        st = r.read_stats()
        assert st["status"] == 0
        assert st["cache_queries"] > 4 * 2048 * 32     # several tiles per wave of the persistent grid
        frames.append(rgb.reshape(-1, 3).double().cpu().numpy())
        del r, cache, rgb
    g, gz = frames
    reached = np.flatnonzero(np.abs(g - gz).max(axis=1) > 1e-3)
    assert len(reached) > 10000
    rng = np.random.default_rng(23)
    others = S.pixel_subset(w.camera, 8, 24)
    pixels = np.unique(np.concatenate([rng.choice(reached, 40, replace=False), others]))
    ref = oracle.render_cache(w.scene, w.camera, w.params, 2, pixels=pixels)
    rec = ref["records"]
    feats = M.encode(rec[:, 1:4], rec[:, 4:7], rec[:, 7:10], bounds[0], bounds[1])
    y, _ = M.forward(ws, feats)
    term = rec[:, 10:13] * np.maximum(y, 0.0) / spp
    img = ref["rgb"].copy()
    cache_mag = np.zeros_like(img)
    np.add.at(img, rec[:, 0].astype(int), term)
    np.add.at(cache_mag, rec[:, 0].astype(int), np.abs(term))
    rob = ref["margin"] > 1e-4
    hit = np.isin(pixels, reached)
    assert (rob & hit).sum() >= 6 and (rob & ~hit).sum() >= 2, (rob & hit).sum()
    err = np.abs(g[pixels] - img).max(axis=1)
    tol = 1e-3 + 3e-2 * cache_mag.max(axis=1)
    assert (err[rob] <= tol[rob]).all(), (err - tol)[rob].max()
    assert (cache_mag[rob & hit].max(axis=1) > 1e-3).sum() >= 4   # the compared pixels carry cache terms


def _poison(cache, key, index, nbytes, dtype, bits):
    view = cache._view(key, nbytes, dtype)
    view[index] = bits
    torch.cuda.synchronize()


def test_unhealthy_cache_falls_back_to_the_plain_tracer(rt):
    """The plain full-depth tracer is the learned form's fallback: a NaN in the BF16 weights a frame is about
    to use makes that frame answer no query and trace on to max_depth instead (the plain frame, reported by
    the status bit); a NaN that enters the FP32 master weights shows in the next frame, after training has
    turned the loss and the weights non-finite.  Initialising the state again restores the learned form."""
    w = _scene()
    sc = rt.Scene(w.scene).upload()
    plain_rgb, plain_ids, _ = rt.render(sc, w.camera, w.params)
    torch.cuda.synchronize()
    cache = rt.RadianceCache(S.mlp_init_weights(5), capacity=2048)
    r = rt.CachedRenderer(sc, w.camera, w.params, cache, mode=rt.CACHE_TRAIN, depth=2, full_depth=w.params.max_depth,
                          train_samples=2048, train_steps=2)
    healthy, _ = r.render(rt.FLAG_SYNC)
    healthy = healthy.clone()
    torch.cuda.synchronize()
    assert r.read_stats()["status"] == 0 and cache.health() == 0
    assert r.read_stats()["cache_queries"] > 50
    assert (healthy - plain_rgb).abs().max() > 1e-3           # the learned frame differs from the plain one

    # (1) a NaN BF16 weight: this very frame falls back (graph replay and eager launches alike)
    n = rt.mlp_num_params()
    _poison(cache, "w_bf16", 4097, 2 * n, torch.int16, 0x7FC0)
    for flags in (rt.FLAG_SYNC, rt.FLAG_SYNC | rt.FLAG_NO_GRAPH):
        rgb, ids = r.render(flags)
        torch.cuda.synchronize()
        st = r.read_stats()
        assert st["status"] == rt.STATUS_CACHE_FALLBACK, st["status"]
        assert st["cache_queries"] == 0
        assert torch.equal(ids, plain_ids)
        assert torch.allclose(rgb, plain_rgb, rtol=1e-5, atol=1e-5), (rgb - plain_rgb).abs().max()
        assert cache.health() & rt.CACHE_HEALTH_BF16
    # the same rays as the plain frame, depth by depth
    r_plain = rt.Renderer(sc, w.camera, w.params)
    r_plain.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    assert r.read_stats()["rays"] == r_plain.read_stats()["rays"]
    assert r.read_stats()["shadow"] == r_plain.read_stats()["shadow"]

    # (2) re-initialised: the learned form is back
    cache2 = rt.RadianceCache(S.mlp_init_weights(5), capacity=2048)
    r2 = rt.CachedRenderer(sc, w.camera, w.params, cache2, mode=rt.CACHE_TRAIN, depth=2,
                           full_depth=w.params.max_depth, train_samples=2048, train_steps=2)
    again, _ = r2.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    assert r2.read_stats()["status"] == 0 and cache2.health() == 0
    assert torch.allclose(again, healthy, rtol=1e-5, atol=1e-5)

    # (3) a NaN master weight: the frame still uses the finite BF16 copy, its training turns the loss and the
    # weights non-finite, and the next frame falls back
    _poison(cache2, "w_master", 123, 4 * n, torch.float32, float("nan"))
    r2.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    assert r2.read_stats()["status"] == 0
    assert cache2.health() & rt.CACHE_HEALTH_WEIGHTS
    rgb, ids = r2.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    assert r2.read_stats()["status"] == rt.STATUS_CACHE_FALLBACK
    assert torch.allclose(rgb, plain_rgb, rtol=1e-5, atol=1e-5)


def test_cache_checkpoint_round_trip(rt, tmp_path):
    """Saving and loading the network's state (master weights, Adam moments, step count) resumes training
    exactly: the next frame of the loaded state equals that of the original, image and weights."""
    w = _scene()
    sc = rt.Scene(w.scene).upload()
    kw = dict(mode=rt.CACHE_TRAIN, depth=2, full_depth=6, train_samples=2048, train_steps=2)
    cache = rt.RadianceCache(S.mlp_init_weights(9), capacity=2048)
    r = rt.CachedRenderer(sc, w.camera, w.params, cache, **kw)
    for f in range(3):
        w.params.frame = f
        r.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    path = str(tmp_path / "cache.npz")
    cache.save(path)
    loaded = rt.RadianceCache.load(path)
    assert loaded.counters()["steps"] == cache.counters()["steps"] == 6
    assert torch.equal(loaded.master_weights(), cache.master_weights())
    assert torch.equal(loaded.bf16_weights(), cache.bf16_weights())
    r_loaded = rt.CachedRenderer(sc, w.camera, w.params, loaded, **kw)
    w.params.frame = 3
    a, _ = r.render(rt.FLAG_SYNC)
    b, _ = r_loaded.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    # the same weights give the same image up to the order of the per-pixel atomic additions
    assert torch.allclose(a, b, rtol=1e-5, atol=1e-6)
    # training is deterministic up to the order of the gradient's atomic additions
    assert torch.allclose(loaded.master_weights(), cache.master_weights(), rtol=0, atol=1e-6)
    assert loaded.counters()["steps"] == 8
