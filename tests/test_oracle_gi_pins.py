"""Pins of the oracle's global illumination (Eq. 8 by path tracing) against closed forms.

Each pin is something the mathematics fixes independently of the oracle's code:
  * inside a closed sphere lit by a point light at its centre every wall point
    has the same local radiance L0 = I k_d a, and every bounce lands on the wall
    again, so the path sum is a geometric series in the bounce factor;
  * the expectation of the randomly chosen branch is the full branching sum
    (mixed diffuse + mirror walls: series in k_d a + k_r);
  * diffuse directions are cosine-distributed: cos^2(theta) and the azimuth are
    uniform;
  * with k_d = 0 everywhere a mirror path has one branch per bounce and equals
    Whitted recursion exactly; with a dielectric its mean converges to it.
"""
import math

import numpy as np

import oracle
from paper_1504_03151_amd import scenes as S

I = 0.75          # light intensity (every constant is exact in FP32)


def _inside_sphere(mat, depth, spp=1, gi=1, eye=(0.25, -0.5, 0.125)):
    sc = S.make_scene(spheres=[[0.0, 0.0, 0.0, 4.0]], sphere_mat=[0], materials=np.stack([mat]),
                      lights=[[0.0, 0.0, 0.0, I, I, I]])
    cam = S.Camera(eye, (1.0, 0.5, 2.0), (0.0, 1.0, 0.0), 90.0, 3, 2)
    p = S.Params(spp=spp, max_depth=depth, jitter=1, seed=5, frame=2, gi=gi)
    return sc, cam, p


def test_diffuse_sphere_interior_is_a_geometric_series():
    """Closed sphere, Lambert walls of colour k_d a, point light at the centre (N.L = 1 on every wall point):
    L = I q (1 + q + ... + q^D), q = k_d a per channel, for every pixel and sample (no variance)."""
    a = np.array([0.75, 0.5, 0.25])
    kd = 0.875
    mat = S.material(tuple(a), k_a=0.0, k_d=kd, k_s=0.0, k_r=0.0)
    for D in (0, 1, 2, 6):
        sc, cam, p = _inside_sphere(mat, D, spp=3)
        out = oracle.render(sc, cam, p)
        q = kd * a
        expect = I * q * sum(q ** j for j in range(D + 1))
        np.testing.assert_allclose(out["rgb_s"].reshape(-1, 3), np.broadcast_to(expect, (6 * 3, 3)), rtol=1e-12)
        # one closed-hit query per depth, one shadow ray per hit
        assert (out["counts"][:, :, 0] == 3).all() and (out["counts"][:, :, 1] == 3).all()
    # Whitted recursion of the same walls has no diffuse bounce: the local term only
    sc, cam, p = _inside_sphere(mat, 6, gi=0)
    np.testing.assert_allclose(oracle.render(sc, cam, p)["rgb"], np.broadcast_to(I * kd * a, (6, 3)), rtol=1e-12)


def test_mixed_diffuse_mirror_walls_converge_to_the_branching_sum():
    """Walls with k_d a (coloured) and k_r: one random branch per bounce; the mean over samples is
    L0 (1 + g + ... + g^D), g = k_d a + k_r per channel."""
    a = np.array([0.75, 0.25, 0.5])
    kd, kr, D = 0.5, 0.375, 4
    mat = S.material(tuple(a), k_a=0.0, k_d=kd, k_s=0.0, k_r=kr)
    sc, cam, p = _inside_sphere(mat, D, spp=2048)
    out = oracle.render(sc, cam, p, pixels=[0, 4])
    g = kd * a + kr
    expect = I * kd * a * sum(g ** j for j in range(D + 1))
    vals = out["rgb_s"].reshape(-1, 3)
    sem = vals.std(0) / math.sqrt(len(vals))
    assert (sem > 0).all()                                    # the branch choice is random
    assert (np.abs(vals.mean(0) - expect) < 5 * sem).all(), (vals.mean(0), expect, sem)
    # the per-sample values are products of the two bounce factors: diffuse k_d a S / m_d, mirror S
    S_ = kd * a.max() + kr
    fd, fr = kd * a * S_ / (kd * a.max()), S_
    L0 = I * kd * a
    ok = np.zeros(len(vals), bool)
    import itertools
    for path in itertools.product((0, 1), repeat=D):
        w, tot = np.ones(3), L0.copy()
        for b in path:
            w = w * (fd if b == 0 else fr)
            tot = tot + w * L0
        ok |= np.abs(vals - tot).max(1) < 1e-12
    assert ok.all()
    # the diffuse branch is taken with probability m_d / S = 0.375 / 0.75
    first = oracle.ray_tree(sc, cam, p, 0, 0)[0]
    kinds = [oracle.ray_tree(sc, cam, p, 0, s)[0][2, 0] for s in range(600)]   # record 2: the depth-1 ray
    assert first[1, 0] == 3                                    # record 1: the primary hit's shadow ray
    frac = np.mean(np.array(kinds) == 4)
    assert abs(frac - 0.5) < 4 * math.sqrt(0.25 / 600), frac


def test_diffuse_directions_are_cosine_distributed():
    """On a Lambert floor: cos(theta) of the bounce direction has P(cos <= c) = c^2 and the azimuth is uniform."""
    mats = np.stack([S.material((0.5, 0.5, 0.5), k_a=0.0, k_d=1.0, k_s=0.0)])
    sc = S.make_scene(planes=[[0.0, 1.0, 0.0, 0.0]], plane_mat=[0], materials=mats,
                      lights=[[0.0, 5.0, 0.0, 1.0, 1.0, 1.0]])
    cam = S.Camera((0.0, 3.0, 0.0), (0.0, 0.0, 0.01), (0.0, 0.0, 1.0), 60.0, 40, 40)
    p = S.Params(spp=3, max_depth=1, jitter=1, seed=9, gi=1)
    cos, phi = [], []
    for pix in range(0, 1600, 1):
        rec = oracle.ray_tree(sc, cam, p, pix, pix % 3)[0]
        rec = rec[rec[:, 0] == 4]
        assert len(rec) == 1 and rec[0, 1] == 1
        d = rec[0, 5:8]
        assert abs(np.linalg.norm(d) - 1.0) < 1e-12
        cos.append(d[1])
        phi.append(math.atan2(d[2], d[0]))
    cos, phi = np.array(cos), np.array(phi)
    n = len(cos)
    assert cos.min() >= 0.0
    ks = 1.63 / math.sqrt(n)                                   # Kolmogorov-Smirnov, 1 %
    x = np.sort(cos ** 2)
    assert np.abs(x - (np.arange(1, n + 1) - 0.5) / n).max() < ks
    y = np.sort((phi + math.pi) / (2 * math.pi))
    assert np.abs(y - (np.arange(1, n + 1) - 0.5) / n).max() < ks
    assert abs(cos.mean() - 2.0 / 3.0) < 5 * math.sqrt(1.0 / 18.0 / n)   # E cos = 2/3, Var cos = 1/18


def _specular_scene(with_glass):
    mats = [S.material((0.75, 0.5, 0.25), k_a=0.25, k_d=0.0, k_s=0.5, k_r=0.5, mtype=S.MIRROR),
            S.material((0.25, 0.5, 0.75), k_a=0.5, k_d=0.0, k_s=0.25, k_r=0.25),
            S.dielectric_material(1.5, k_s=0.5)]
    spheres = [[-1.0, 1.0, 0.0, 1.0], [1.25, 0.75, 0.5, 0.75]]
    return S.make_scene(spheres=spheres, sphere_mat=[0, 2 if with_glass else 1], planes=[[0.0, 1.0, 0.0, 0.0]],
                        plane_mat=[1], materials=np.stack(mats), lights=[[2.0, 6.0, -3.0, 1.0, 1.0, 1.0]])


def test_without_diffuse_terms_a_path_is_whitted_recursion():
    sc = _specular_scene(with_glass=False)
    cam = S.Camera((0.0, 2.0, -6.0), (0.0, 0.75, 0.0), (0.0, 1.0, 0.0), 45.0, 24, 16)
    p = S.Params(spp=2, max_depth=6, jitter=1, seed=3)
    whitted = oracle.render(sc, cam, p)
    p.gi = 1
    path = oracle.render(sc, cam, p)
    assert np.array_equal(path["rgb_s"], whitted["rgb_s"])
    assert np.array_equal(path["counts"], whitted["counts"])


def test_dielectric_paths_average_to_whitted_recursion():
    """A glass sphere: a path takes the reflected or the refracted branch with probability F or 1 - F and
    factor 1; over many passes through the same camera ray the mean is the Whitted radiance."""
    sc = _specular_scene(with_glass=True)
    cam = S.Camera((0.0, 2.0, -6.0), (1.25, 0.75, 0.5), (0.0, 1.0, 0.0), 10.0, 3, 3)
    K = 3001                                                  # not a square: every sample through the centre
    p = S.Params(spp=K, max_depth=5, jitter=0, seed=4)
    whitted = oracle.render(sc, cam, p, pixels=[4])
    assert whitted["ids"][0, 0] == 1                          # the glass sphere
    p.gi = 1
    vals = oracle.render(sc, cam, p, pixels=[4])["rgb_s"][0]
    sem = vals.std(0) / math.sqrt(K)
    assert (sem > 0).all()
    assert (np.abs(vals.mean(0) - whitted["rgb"][0]) < 5 * sem).all(), (vals.mean(0), whitted["rgb"][0], sem)


def test_path_random_numbers_are_uniform_and_keyed():
    u = np.array([oracle.path_rand(1, 2, p, 3, 4, 0) for p in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert (u * 2 ** 24 == np.floor(u * 2 ** 24)).all()       # 24 bits, exact in FP32
    n = len(u)
    x = np.sort(u)
    assert np.abs(x - (np.arange(1, n + 1) - 0.5) / n).max() < 1.63 / math.sqrt(n)
    base = oracle.path_rand(1, 2, 5, 3, 4, 0)
    for args in ((1, 2, 5, 3, 4, 1), (1, 2, 5, 3, 5, 0), (1, 2, 5, 4, 4, 0), (1, 3, 5, 3, 4, 0), (2, 2, 5, 3, 4, 0)):
        assert oracle.path_rand(*args) != base
    assert oracle.path_rand(1, 2, 5, 3, 4, 0) != oracle.jitter(1, 2, 5, 3, 0)


def test_cut_off_plus_keyed_depth2_paths_is_the_full_path_traced_render():
    """A path is linear in what its depth-2 ray returns: the image cut off at depth 2 plus, for every depth-2
    hit, its path weight times the radiance of a path restarted there with the same pixel key (and sample)
    equals the full path-traced image.  Pins the cut-off and the keying of the learned form's targets."""
    w = S.random_tiny(11, size=40, depth=5)
    w.camera.height = 37
    w.params.gi = 1
    assert w.params.spp == 1
    full = oracle.render(w.scene, w.camera, w.params)
    cut = oracle.render_cache(w.scene, w.camera, w.params, 2)
    rec = cut["records"]
    assert len(rec) > 30
    x, v, wt = rec[:, 1:4], rec[:, 7:10], rec[:, 10:13]
    d = -v
    idx = rec[:, 0].astype(int)
    L, m = oracle.radiance(w.scene, w.params, x - 1e-2 * d, d, 2, pixels=idx, sample=0)
    recon = cut["rgb"].copy()
    np.add.at(recon, idx, wt * L)
    ok = (full["margin"] > 1e-4) & (cut["margin"] > 1e-4)
    bad = np.zeros(len(ok), bool)
    bad[idx[m <= 1e-4]] = True
    ok &= ~bad
    assert ok.mean() > 0.9
    np.testing.assert_allclose(recon[ok], full["rgb"][ok], rtol=0, atol=1e-9)
    touched = np.zeros(len(ok), bool)
    touched[idx] = True
    assert (np.abs(full["rgb"] - cut["rgb"]).max(axis=1)[ok & touched] > 1e-6).sum() > 20
    # another key draws another continuation
    L2, _ = oracle.radiance(w.scene, w.params, x - 1e-2 * d, d, 2, pixels=idx + 1, sample=0)
    assert np.abs(L2 - L).max() > 1e-3
