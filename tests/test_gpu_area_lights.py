"""Area lights sampled once per pass (the paper's progressive scheme, Section V) on the GPU against the oracle.

Both sides draw the same sample point of each light for each pass from the counter hash, so images are
compared pixel by pixel like point-lit ones (ids exact and RGB within 1e-3 on robust pixels); the pass
average is also checked against the closed-form shadow of a sphere under a disk light.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1504_03151_amd import scenes as S

pytestmark = pytest.mark.gpu
ROBUST = 1e-4
RGB_TOL = 1e-3


@pytest.fixture(scope="module")
def rt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_03151_amd import rt as _rt
    _rt.lib()
    return _rt


def area_tiny(seed, size=40):
    """A tiny mixed scene whose two lights are a disk and a parallelogram."""
    w = S.random_tiny(seed, size=size, depth=3)
    L = w.scene.lights.copy()
    L[0, 6], L[0, 7:10], L[0, 10:13] = S.DISK, [1.5, 0.0, 0.0], [0.0, 0.0, 1.5]
    L[1, 6], L[1, 7:10], L[1, 10:13] = S.PARALLELOGRAM, [2.0, 0.0, 0.0], [0.0, 0.5, 1.0]
    w.scene.lights = L
    w.params.spp, w.params.jitter = 4, 1
    return w


@pytest.mark.parametrize("seed", [0, 3])
def test_area_lit_tiny_scene_every_pixel(rt, seed):
    w = area_tiny(seed)
    sc = rt.Scene(w.scene).upload()
    rgb, ids, st = rt.render(sc, w.camera, w.params)
    torch.cuda.synchronize()
    ref = oracle.render(w.scene, w.camera, w.params)
    rob = ref["margin"] > ROBUST
    assert rob.mean() > 0.965                              # oracle: 0.9762 (seed 0), 0.9725 (seed 3)
    g_ids = ids.reshape(-1, w.params.spp).cpu().numpy()
    assert (g_ids[rob] == ref["ids"][rob]).all()
    err = np.abs(rgb.reshape(-1, 3).double().cpu().numpy() - ref["rgb"]).max(axis=1)
    assert err[rob].max() <= RGB_TOL, err[rob].max()
    # another frame samples other light points: the image changes where the lights are visible
    w.params.frame = 1
    rgb1, _, _ = rt.render(sc, w.camera, w.params)
    torch.cuda.synchronize()
    ref1 = oracle.render(w.scene, w.camera, w.params)
    assert np.abs(ref1["rgb"] - ref["rgb"]).max() > 1e-2
    err1 = np.abs(rgb1.reshape(-1, 3).double().cpu().numpy() - ref1["rgb"]).max(axis=1)
    rob1 = ref1["margin"] > ROBUST
    assert err1[rob1].max() <= RGB_TOL


def test_disk_light_pass_average_matches_the_closed_form(rt):
    D, R, a, r = 4.0, 2.0, 2.0, 0.5
    mats = np.stack([S.material((1.0, 1.0, 1.0), k_a=0.0, k_d=1.0, k_s=0.0, k_r=0.0),
                     S.material((0.5, 0.5, 0.5), k_a=0.0, k_d=1.0, k_s=0.0, k_r=0.0)])
    scene = S.make_scene(spheres=[[0.0, a, 0.0, r]], sphere_mat=[1], planes=[[0.0, 1.0, 0.0, 0.0]], plane_mat=[0],
                         materials=mats, lights=[[0.0, D, 0.0, 1.0, 1.0, 1.0, S.DISK, R, 0.0, 0.0, 0.0, 0.0, R]])
    cam = S.Camera((6.0, 2.0, 0.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 1, 1)
    K = 4095
    p = S.Params(spp=K, max_depth=0, jitter=0, seed=11)
    sc = rt.Scene(scene).upload()
    rgb, ids, st = rt.render(sc, cam, p, per_sample=True)
    torch.cuda.synchronize()
    vals = rgb.reshape(K, 3)[:, 0].double().cpu().numpy()
    e = 1e-3
    rho0 = (D - e) * math.tan(math.asin(r / (a - e)))
    expect = 2.0 * D / R ** 2 * (math.sqrt(D * D + R * R) - math.sqrt(D * D + rho0 * rho0))
    assert abs(vals.mean() - expect) < 4.0 * vals.std() / math.sqrt(K), (vals.mean(), expect)
    ref = oracle.render(scene, cam, p)
    rob = ref["margin_s"][0] > ROBUST
    assert rob.mean() > 0.99
    assert np.abs(vals - ref["rgb_s"][0, :, 0])[rob].max() <= RGB_TOL
    assert st["shadow"][0] == K


def test_batch_with_area_lights_equals_sequential_frames(rt):
    ws = [area_tiny(0, size=24), S.random_tiny(5, size=20), area_tiny(3, size=31)]
    scs = [rt.Scene(w.scene).upload() for w in ws]
    br = rt.BatchRenderer(scs, [w.camera for w in ws], [w.params for w in ws])
    rgb_b, ids_b = br.render(rt.FLAG_SYNC)
    torch.cuda.synchronize()
    for w, sc, rb, ib in zip(ws, scs, rgb_b, ids_b):
        rgb, ids, _ = rt.render(sc, w.camera, w.params)
        torch.cuda.synchronize()
        assert torch.equal(ids, ib)
        assert torch.allclose(rgb, rb, rtol=1e-5, atol=1e-6), (rgb - rb).abs().max().item()


def test_progressive_passes_average_the_frames(rt):
    """Progressive mode (the paper's pass-by-pass image update): frame f added to the f frames already in the
    accumulator gives the mean of frames 0..f, also through graph replays; the mean of the area-lit passes
    matches the oracle's mean of the same passes."""
    w = area_tiny(0, size=32)
    w.params.spp, w.params.jitter = 1, 1
    sc = rt.Scene(w.scene).upload()
    single = rt.Renderer(sc, w.camera, w.params)
    prog = rt.Renderer(sc, w.camera, w.params)
    frames = []
    for f in range(6):
        w.params.frame = f
        img, _ = single.render(rt.FLAG_SYNC)
        frames.append(img.clone())
        acc, _ = prog.render(rt.FLAG_SYNC, accum_frames=f)
        torch.cuda.synchronize()
        expect = torch.stack(frames).mean(0)
        assert torch.allclose(acc, expect, rtol=1e-5, atol=1e-6), (f, (acc - expect).abs().max().item())
    refs = []
    for f in range(6):
        w.params.frame = f
        refs.append(oracle.render(w.scene, w.camera, w.params))
    rob = np.all([r["margin"] > ROBUST for r in refs], axis=0)
    assert rob.mean() > 0.965                              # oracle: 0.9717 (robust in all six frames)
    ref_mean = np.mean([r["rgb"] for r in refs], axis=0)
    err = np.abs(acc.reshape(-1, 3).double().cpu().numpy() - ref_mean).max(axis=1)
    assert err[rob].max() <= RGB_TOL
    # starting afresh discards the accumulator
    w.params.frame = 2
    again, _ = prog.render(rt.FLAG_SYNC, accum_frames=0)
    torch.cuda.synchronize()
    assert torch.allclose(again, frames[2], rtol=1e-5, atol=1e-6)
