"""Pins of the FP64 oracle against closed forms, invariants and special cases.

Nothing here compares the oracle with itself: every expected value is derived
by hand from geometry or optics (written out next to each case), or is a
property any correct tracer has (permutation invariance, mirror symmetry,
linearity).  The paper fixes the sphere quadratic (Eq. 9-12, Section IV.B),
the brute-force object loop and the blocker loop (Algorithm 1, Section III)
and the recursive secondary rays (Section III, IV.A, Fig. 3).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1504_03151_amd import scenes as S

CAP = 1e-2


def _scene(**kw):
    kw.setdefault("materials", np.stack([S.material((0.8, 0.3, 0.2))]))
    kw.setdefault("lights", [[0.0, 10.0, 0.0, 1.0, 1.0, 1.0]])
    return S.make_scene(**kw)


# ---------------------------------------------------------------- spheres (Eq. 11-12)

def test_sphere_roots_closed_form():
    sc = _scene(spheres=[[0.0, 0.0, 0.0, 1.0], [1.0, 2.0, 3.0, 2.0]], sphere_mat=[0, 0])
    o = [[0, 0, -10], [0, 0.5, -10], [0, 0, 0], [0, -1.5, -10], [0, 0, -10], [1, 2, -10]]
    d = [[0, 0, 1], [0, 0, 1], [0, 0, 1], [0, 0, 1], [0, 0, -1], [0, 0, 1]]
    t, ids, m = oracle.closest(sc, o, d)
    # a=1, b=2(o-c).d, c'=|o-c|^2-r^2: t=(-b-sqrt(b^2-4c'))/2
    assert t[0] == 9.0 and ids[0] == 0                      # b=-20, c'=99 -> t=(20-2)/2
    assert abs(t[1] - (10.0 - math.sqrt(0.75))) < 1e-12 and ids[1] == 0
    assert t[2] == 1.0 and ids[2] == 0                      # origin inside: far root
    assert ids[3] == -1 and np.isinf(t[3])                  # |o_perp| = 1.5 > r
    assert ids[4] == -1                                     # sphere behind the ray
    assert t[5] == 11.0 and ids[5] == 1                     # r=2 sphere at z=3, from z=-10


def test_sphere_tangent_is_not_robust():
    sc = _scene(spheres=[[0.0, 0.0, 0.0, 1.0]], sphere_mat=[0])
    t, ids, m = oracle.closest(sc, [[0, 1.0, -10]], [[0, 0, 1]])
    assert ids[0] == 0 and t[0] == 10.0 and m[0] < 1e-4      # tangent: hit with zero margin
    t, ids, m = oracle.closest(sc, [[0, 0.0, -10]], [[0, 0, 1]])
    assert m[0] == CAP                                       # central hit: clearly robust


def test_plane_closed_form():
    sc = _scene(planes=[[0.0, 1.0, 0.0, -5.0]], plane_mat=[0])
    s2 = 1 / math.sqrt(2)
    t, ids, m = oracle.closest(sc, [[0, 0, 0], [0, 0, 0], [0, 0, 0]], [[0, -1, 0], [0, -s2, s2], [0, 1, 0]])
    assert t[0] == 5.0 and ids[0] == 0
    assert abs(t[1] - 5 * math.sqrt(2)) < 1e-12
    assert ids[2] == -1


# ---------------------------------------------------------------- triangles

TRI = [[-1.0, -1.0, 5.0], [1.0, -1.0, 5.0], [0.0, 1.0, 5.0]]


def test_hit_surface_coordinates():
    # triangle: aiming at (1-u-v) v0 + u v1 + v v2 returns (u, v); the centroid returns (1/3, 1/3);
    # a vertex returns its own unit weight
    v0, v1, v2 = (np.array(v, np.float64) for v in TRI)
    targets = [(0.2, 0.3), (1 / 3, 1 / 3), (0.0, 1.0), (0.7, 0.05)]
    o, d = [], []
    for u, v in targets:
        x = (1 - u - v) * v0 + u * v1 + v * v2
        src = np.array([0.3, -0.2, -4.0])
        dd = x - src
        o.append(src)
        d.append(dd / np.linalg.norm(dd))
    sc = _scene(tris=[TRI], tri_mat=[0])
    t, ids, m, uv = oracle.closest(sc, o, d, uv=True)
    assert (ids == 0).all()
    np.testing.assert_allclose(uv, np.array(targets), rtol=0, atol=1e-12)
    # sphere: unit sphere at the origin; u = (atan2(n_z, n_x) + pi) / (2 pi), v = acos(n_y) / pi
    sc = _scene(spheres=[[0.0, 0.0, 0.0, 1.0]], sphere_mat=[0])
    th, ph = 1.1, 0.4                                        # hit normal n = (sin th cos ph, cos th, sin th sin ph)
    n = np.array([math.sin(th) * math.cos(ph), math.cos(th), math.sin(th) * math.sin(ph)])
    o = [[0, 0, -10], [10, 0, 0], [0, 10, 0], list(5 * n)]
    d = [[0, 0, 1], [-1, 0, 0], [0, -1, 0], list(-n)]
    t, ids, m, uv = oracle.closest(sc, o, d, uv=True)
    assert (ids == 0).all()
    expect = [(0.25, 0.5),                                   # n = (0, 0, -1): atan2(-1, 0) = -pi/2
              (0.5, 0.5),                                    # n = (1, 0, 0): atan2(0, 1) = 0
              (None, 0.0),                                   # the pole n = +y: polar angle 0
              ((ph + math.pi) / (2 * math.pi), th / math.pi)]
    for (eu, ev), (gu, gv) in zip(expect, uv):
        if eu is not None:
            assert abs(gu - eu) < 1e-12
        assert abs(gv - ev) < 1e-7
    # planes and misses carry (0, 0)
    sc = _scene(planes=[[0.0, 1.0, 0.0, -5.0]], plane_mat=[0])
    _, ids, _, uv = oracle.closest(sc, [[0, 0, 0], [0, 0, 0]], [[0, -1, 0], [0, 1, 0]], uv=True)
    assert ids[0] == 0 and ids[1] == -1 and (uv == 0).all()


def test_triangle_hit_edges_inclusive_and_degenerate():
    sc = _scene(tris=[TRI], tri_mat=[0])
    o = [[0, 0, 0], [-1, -1, 0], [-1.001, -1, 0], [0, 1, 0], [0, 1.0001, 0], [0, 0, 6]]
    d = [[0, 0, 1]] * 5 + [[0, 0, 1]]
    t, ids, m = oracle.closest(sc, o, d)
    assert t[0] == 5.0 and ids[0] == 0
    assert m[0] == CAP                      # barycentrics (0.25, 0.25, 0.5): far from every edge
    assert ids[1] == 0 and m[1] < 1e-4      # exactly through a vertex: hit, not robust
    assert ids[2] == -1
    assert ids[3] == 0 and m[3] < 1e-4      # apex
    assert ids[4] == -1
    assert ids[5] == -1                     # triangle behind the origin
    deg = _scene(tris=[[[0, 0, 5], [1, 1, 5], [2, 2, 5]]], tri_mat=[0])   # zero area
    _, ids, _ = oracle.closest(deg, [[1, 1, 0]], [[0, 0, 1]])
    assert ids[0] == -1


def test_quad_is_watertight_and_ties_go_to_smaller_id():
    a, b, c, d_ = [0, 0, 5], [1, 0, 5], [1, 1, 5], [0, 1, 5]
    sc = _scene(tris=[[a, b, c], [a, c, d_]], tri_mat=[0, 0])
    rng = np.random.default_rng(0)
    x = rng.uniform(0.001, 0.999, 400)
    o = np.stack([x, x, np.zeros_like(x)], 1)                        # through the shared diagonal
    t, ids, _ = oracle.closest(sc, o, np.tile([0.0, 0.0, 1.0], (400, 1)))
    assert (ids == 0).all() and (t == 5.0).all()                    # both accept; tie -> smaller id
    p = rng.uniform(0.001, 0.999, (2000, 2))
    o = np.concatenate([p, np.zeros((2000, 1))], 1)
    t, ids, _ = oracle.closest(sc, o, np.tile([0.0, 0.0, 1.0], (2000, 1)))
    assert (ids >= 0).all()
    assert ((ids == 0) == (p[:, 0] >= p[:, 1])).all()


def test_closest_hit_is_invariant_under_primitive_permutation():
    w = S.random_tiny(3, n_spheres=5, n_tris=40)
    sc = w.scene
    rng = np.random.default_rng(1)
    o = rng.uniform(-6, 6, (300, 3))
    dvec = rng.normal(size=(300, 3))
    dvec /= np.linalg.norm(dvec, axis=1, keepdims=True)
    t, ids, m = oracle.closest(sc, o, dvec)
    ps, pt = rng.permutation(len(sc.spheres)), rng.permutation(len(sc.tris))
    sc2 = S.make_scene(spheres=sc.spheres[ps], sphere_mat=sc.sphere_mat[ps], tris=sc.tris[pt],
                       tri_mat=sc.tri_mat[pt], planes=sc.planes, plane_mat=sc.plane_mat,
                       materials=sc.materials, lights=sc.lights)
    t2, ids2, _ = oracle.closest(sc2, o, dvec)
    ns = len(sc.spheres)
    new_to_old = np.concatenate([ps, ns + pt, ns + len(pt) + np.arange(len(sc.planes))])
    mapped = np.where(ids2 >= 0, new_to_old[np.maximum(ids2, 0)], -1)
    robust = m > 1e-4
    assert robust.mean() > 0.95
    assert (mapped[robust] == ids[robust]).all()
    assert np.allclose(t2[robust], t[robust], rtol=0, atol=0)


# ---------------------------------------------------------------- camera

def test_camera_corner_directions_closed_form():
    w = S.config0()
    cam, p = w.camera, w.params
    o, d = oracle.camera_rays(cam, p, [0, 127, 127 * 128 + 127])
    th = math.tan(math.radians(30.0))
    for dd, (sx, sy) in zip(d, [(-1, 1), (1, 1), (1, -1)]):
        e = np.array([sx * (1 - 1 / 128) * th, sy * (1 - 1 / 128) * th, 1.0])   # f=(0,0,1), r=+x, u=+y
        assert np.allclose(dd, e / np.linalg.norm(e), atol=1e-15)
    assert np.allclose(o, [[0, 0, -10]] * 3)


def test_stratified_jitter_stays_in_its_stratum():
    w = S.config2(width=32, height=18, n_objects=2, subdivisions=0)
    cam, p = w.camera, w.params
    th = math.tan(math.radians(30.0))
    aspect = cam.width / cam.height
    pix = 5 * 32 + 7
    for s in range(16):
        _, d = oracle.camera_rays(cam, p, [pix], sample=s)
        X, Y = d[0, 0] / d[0, 2], d[0, 1] / d[0, 2]           # f=(0,0,1): image-plane coordinates
        jx = ((X / (aspect * th)) + 1) * cam.width / 2 - 7
        jy = (1 - Y / th) * cam.height / 2 - 5
        assert (s % 4) / 4 <= jx < (s % 4 + 1) / 4 + 1e-12
        assert (s // 4) / 4 <= jy < (s // 4 + 1) / 4 + 1e-12


def test_jitter_hash_uniform_and_bijective():
    xs = np.array([oracle.jitter(7, 0, i, 3, 0) for i in range(20000)])
    assert xs.min() >= 0 and xs.max() < 1
    hist = np.histogram(xs, bins=20, range=(0, 1))[0]
    chi2 = ((hist - 1000.0) ** 2 / 1000.0).sum()
    assert chi2 < 45.3                     # 19 dof, p = 0.001
    assert np.all(xs * 2 ** 24 == np.floor(xs * 2 ** 24))   # 24-bit values, exact in FP32
    vals = {oracle.pcg(i) for i in range(1 << 16)}
    assert len(vals) == 1 << 16            # the PCG output permutation is a bijection


# ---------------------------------------------------------------- silhouette and shadows

def test_one_sphere_silhouette_closed_form():
    c, r = np.array([0.3, -0.2, 0.5]), 1.3
    w = S.one_sphere(center=tuple(c), radius=r, size=48)
    out = oracle.render(w.scene, w.camera, w.params)
    o, d = oracle.camera_rays(w.camera, w.params, np.arange(48 * 48))
    dist = np.linalg.norm(np.cross(c - o, d), axis=1)      # distance of the ray line from the centre
    expect = dist < r
    robust = out["margin"] > 1e-4
    assert robust.mean() > 0.98
    assert ((out["ids"][:, 0] == 0) == expect)[robust].all()
    assert expect.sum() > 50


def test_shadow_boundary_closed_form():
    c, r = np.array([0.0, 0.0, 0.0]), 1.5
    light = np.array([2.0, 8.0, -3.0])
    w = S.one_sphere(center=tuple(c), radius=r, plane_y=-3.0, light=tuple(light), size=48)
    w.camera = S.Camera((0.0, 3.0, -12.0), (0.0, -2.0, 0.0), (0.0, 1.0, 0.0), 60.0, 48, 48)
    out = oracle.render(w.scene, w.camera, w.params)
    o, d = oracle.camera_rays(w.camera, w.params, np.arange(48 * 48))
    on_plane = out["ids"][:, 0] == 1
    t = (-3.0 - o[:, 1]) / d[:, 1]
    X = o + t[:, None] * d
    seg = light - X
    u = np.clip(np.einsum("ij,ij->i", c - X, seg) / np.einsum("ij,ij->i", seg, seg), 0, 1)
    dist = np.linalg.norm(X + u[:, None] * seg - c, axis=1)   # distance of segment X->L from the centre
    shadowed = dist < r
    far = np.abs(dist - r) > 1e-2
    sel = on_plane & far & (out["margin"] > 1e-4)
    amb = float(np.float32(0.1)) * 0.75       # material constants are FP32 inputs
    got_shadow = np.all(np.abs(out["rgb"] - amb) < 1e-12, axis=1)
    assert sel.sum() > 300 and shadowed[sel].sum() > 20
    assert (got_shadow[sel] == shadowed[sel]).all()


# ---------------------------------------------------------------- local illumination (Phong)

def _on_axis(mat, light, depth=0):
    w = S.one_sphere(center=(0.0, 0.0, 0.0), radius=1.0, light=light, size=65, mat=mat)
    w.params.max_depth = depth
    pix = 32 * 65 + 32                       # pixel centre exactly on the optical axis
    return oracle.render(w.scene, w.camera, w.params, [pix])["rgb"][0]


ALB = np.array([0.75, 0.25, 0.5])      # exact in FP32, like every constant below


def _close(got, expect, atol=1e-14):
    np.testing.assert_allclose(got, expect, rtol=0, atol=atol)


def test_phong_head_on_light():
    got = _on_axis(S.material(tuple(ALB), k_a=0.125, k_d=1.0, k_s=0.5), (0.0, 0.0, -10.0))
    # hit (0,0,-1): N = L = R = V = (0,0,-1), so N.L = R.V = 1
    _close(got, 0.125 * ALB + ALB + 0.5)


def test_lambert_cosine_at_sixty_degrees():
    # light 8 units from the hit point (0,0,-1), 60 degrees off the normal: (0, 4 sqrt3, -5)
    light = (0.0, float(np.float32(4 * math.sqrt(3))), -5.0)
    got = _on_axis(S.material(tuple(ALB), k_a=0.125, k_d=1.0, k_s=0.5), light)
    L = np.array(light) - [0, 0, -1.0]
    cos = L[2] * -1 / np.linalg.norm(L)                      # N.L, = 1/2 up to the FP32 light position
    assert abs(cos - 0.5) < 1e-7
    # R = 2(N.L)N - L has R.V = N.L for V = N, so spec = 0.5 * cos^32
    _close(got, 0.125 * ALB + cos * ALB + 0.5 * cos ** 32)


def test_phong_specular_lobe_thirty_degrees():
    light = (5.0, 0.0, float(np.float32(-1 - 10 * math.cos(math.radians(30)))))
    got = _on_axis(S.material((0.75, 0.25, 0.5), k_a=0.0, k_d=0.0, k_s=1.0, shininess=32), light)
    L = np.array(light) - [0, 0, -1.0]
    L /= np.linalg.norm(L)                                     # (sin 30, 0, -cos 30) up to FP32 rounding
    # with V = N = (0,0,-1): R = 2(N.L)N - L = (-L_x, 0, L_z), so R.V = -L_z = cos 30
    rv = -L[2]
    assert abs(rv - math.cos(math.radians(30))) < 1e-7
    _close(got, np.full(3, rv ** 32))


def test_light_on_the_back_side_gives_ambient_only_and_no_shadow_ray():
    w = S.one_sphere(center=(0.0, 0.0, 0.0), radius=1.0, light=(0.0, 0.0, 10.0), size=65,
                     mat=S.material(tuple(ALB), k_a=0.125))
    out = oracle.render(w.scene, w.camera, w.params, [32 * 65 + 32])
    _close(out["rgb"][0], 0.125 * ALB, atol=0)
    assert out["counts"][0].tolist() == [[1, 0]]


def test_miss_returns_background():
    w = S.one_sphere(size=16)
    w.params.bg = (0.25, 0.5, 0.75)
    out = oracle.render(w.scene, w.camera, w.params, [0])
    assert out["ids"][0, 0] == -1
    _close(out["rgb"][0], [0.25, 0.5, 0.75], atol=0)


def test_direct_light_is_linear_in_intensity():
    w = S.config0()
    w.scene.materials[:, 3] = 0.0            # no ambient
    w.params.bg = (0.0, 0.0, 0.0)
    pix = S.pixel_subset(w.camera, 300, 1)
    a = oracle.render(w.scene, w.camera, w.params, pix)
    w.scene.lights[:, 3:6] *= 2.0
    b = oracle.render(w.scene, w.camera, w.params, pix)
    np.testing.assert_allclose(b["rgb"], 2.0 * a["rgb"], rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------- recursion: mirror, Fresnel, refraction

def test_plane_mirror_equals_mirror_image_scene():
    mirror = S.material((1, 1, 1), k_a=0.0, k_d=0.0, k_s=0.0, k_r=1.0, mtype=S.MIRROR)
    ball = S.material((0.2, 0.7, 0.4), k_r=0.0)
    cam = S.Camera((0.0, 1.0, -10.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, 40, 40)
    A = S.make_scene(spheres=[[0.0, 2.0, 0.0, 1.0]], sphere_mat=[0], planes=[[0, 1, 0, 0]], plane_mat=[1],
                     materials=np.stack([ball, mirror]), lights=[[3.0, 8.0, -4.0, 1, 1, 1]])
    B = S.make_scene(spheres=[[0.0, -2.0, 0.0, 1.0]], sphere_mat=[0], materials=np.stack([ball]),
                     lights=[[3.0, -8.0, -4.0, 1, 1, 1]])
    # a tiny origin offset keeps the mirrored ray within 1e-8 of the straight one in B
    pa, pb = S.Params(max_depth=1, eps=1e-9), S.Params(max_depth=0, eps=1e-9)
    ra = oracle.render(A, cam, pa)
    rb = oracle.render(B, cam, pb)
    # (with such an offset the FP32 robustness margins are meaningless; this is an FP64-only identity)
    via_mirror = ra["ids"][:, 0] == 1
    assert via_mirror.sum() > 500
    hits_image = via_mirror & (rb["ids"][:, 0] == 0)
    assert hits_image.sum() > 20
    _close(ra["rgb"][via_mirror], rb["rgb"][via_mirror], atol=1e-6)


def test_schlick_normal_incidence_r0():
    glass = S.material((1, 1, 1), k_a=0.0, k_d=0.0, k_s=0.0, ior=1.5, mtype=S.DIELECTRIC)
    w = S.one_sphere(center=(0.0, 0.0, 0.0), radius=1.0, size=65, mat=glass)
    w.params.max_depth = 1
    w.params.bg = (0.25, 0.5, 0.75)
    rgb = oracle.render(w.scene, w.camera, w.params, [32 * 65 + 32])["rgb"][0]
    # F = ((n-1)/(n+1))^2 = 0.04 to the background; the transmitted ray ends at depth 1 with local = 0
    _close(rgb, 0.04 * np.array([0.25, 0.5, 0.75]), atol=1e-15)


# Dielectric interface between two planes: the glass plane y = 0 (Schlick-weighted
# reflection and refraction, ior 1.5, no local terms) and a plane y = -1 whose only
# term is k_a * albedo = C (no lights).  A single camera ray along the optical axis
# of a 65 x 65 image meets y = 0 at a chosen angle; max depth 1, so each secondary
# ray returns either the background or C.
BG = np.array([0.25, 0.5, 0.75])
C_LOW = np.array([1.0, 0.125, 0.5])


def _interface(eye, look_at):
    glass = S.material((1, 1, 1), k_a=0.0, k_d=0.0, k_s=0.0, ior=1.5, mtype=S.DIELECTRIC)
    low = S.material(tuple(C_LOW), k_a=1.0, k_d=0.0, k_s=0.0, k_r=0.0)
    sc = S.make_scene(planes=[[0.0, 1.0, 0.0, 0.0], [0.0, 1.0, 0.0, -1.0]], plane_mat=[0, 1],
                      materials=np.stack([glass, low]))
    cam = S.Camera(eye, look_at, (0.0, 1.0, 0.0), 60.0, 65, 65)
    p = S.Params(max_depth=1, bg=tuple(BG))
    rec, rgb = oracle.ray_tree(sc, cam, p, 32 * 65 + 32)
    return rec, rgb


def test_schlick_entering_at_sixty_degrees():
    # ray from above at 60 degrees to the normal: cos = 1/2 on the air side,
    # F = 0.04 + 0.96 (1 - 1/2)^5 = 0.04 + 0.03 = 0.07 on the reflected ray (background)
    # and 1 - F = 0.93 on the transmitted ray, which reaches the lower plane (C)
    th = math.radians(60)
    rec, rgb = _interface((-10 * math.sin(th), 10 * math.cos(th), 0.0), (0.0, 0.0, 0.0))
    _close(rgb, 0.07 * BG + 0.93 * C_LOW, atol=1e-12)
    # Snell: the transmitted ray leaves the normal at asin(sin 60 / 1.5)
    tr = rec[(rec[:, 0] == 2) & (rec[:, 1] == 1)]
    assert len(tr) == 1
    st = math.sin(th) / 1.5
    _close(tr[0, 5:8], [st, -math.sqrt(1 - st * st), 0.0], atol=1e-12)


def test_schlick_leaving_glass_uses_the_air_side_cosine():
    # ray inside the glass (below y = 0, going up) at sin(theta_i) = 1/sqrt(3):
    # k^2 = 1 - 1.5^2 (1 - 2/3) = 1/4, so the air-side cosine is 1/2 (60 degrees out)
    # and F = 0.07 again; with the glass-side cosine sqrt(2/3) F would be
    # 0.04 + 0.96 (1 - 0.8165)^5 = 0.0402.  The reflected ray goes down to C,
    # the transmitted one up to the background.
    si = 1 / math.sqrt(3)
    ci = math.sqrt(2.0 / 3.0)
    eye = (-0.5 * si / ci, -0.5, 0.0)
    rec, rgb = _interface(eye, (0.0, 0.0, 0.0))
    _close(rgb, 0.07 * C_LOW + 0.93 * BG, atol=1e-12)
    tr = rec[(rec[:, 0] == 2) & (rec[:, 1] == 1)]
    assert len(tr) == 1
    _close(tr[0, 5:8], [math.sqrt(3) / 2, 0.5, 0.0], atol=1e-12)      # 60 degrees from the normal in air


def test_total_internal_reflection_reflects_everything():
    # inside the glass at 60 degrees: sin = 0.866 > 1/1.5, k^2 = 1 - 2.25 * 0.75 < 0:
    # F = 1, no transmitted ray, all of the radiance comes from the reflected ray (C)
    th = math.radians(60)
    eye = (-0.5 * math.tan(th), -0.5, 0.0)
    rec, rgb = _interface(eye, (0.0, 0.0, 0.0))
    _close(rgb, C_LOW, atol=1e-12)
    assert ((rec[:, 0] == 2)).sum() == 0
    assert ((rec[:, 0] == 1) & (rec[:, 1] == 1)).sum() == 1
    # the critical angle asin(2/3) separates the two cases
    for s, transmits in [(0.66, True), (0.67, False)]:
        c = math.sqrt(1 - s * s)
        rec, _ = _interface((-0.5 * s / c, -0.5, 0.0), (0.0, 0.0, 0.0))
        assert ((rec[:, 0] == 2).sum() == 1) == transmits


def test_phong_reflection_weight_k_r():
    # head-on light, k_r = 0.3: local (as in the head-on pin) + 0.3 x the reflected ray,
    # which leaves (0,0,-1) along -z and returns the background
    mat = S.material(tuple(ALB), k_a=0.125, k_d=1.0, k_s=0.5, k_r=0.3)
    w = S.one_sphere(center=(0.0, 0.0, 0.0), radius=1.0, light=(0.0, 0.0, -10.0), size=65, mat=mat)
    w.params.max_depth = 1
    w.params.bg = tuple(BG)
    got = oracle.render(w.scene, w.camera, w.params, [32 * 65 + 32])["rgb"][0]
    _close(got, 0.125 * ALB + ALB + 0.5 + float(np.float32(0.3)) * BG)    # k_r is stored in FP32


def test_ball_lens_on_axis_and_snell_deviation():
    glass = S.material((1, 1, 1), k_a=0.0, k_d=0.0, k_s=0.0, ior=1.5, mtype=S.DIELECTRIC)
    w = S.one_sphere(center=(0.0, 0.0, 0.0), radius=1.0, size=65, mat=glass)
    w.params.max_depth = 3
    rec, _ = oracle.ray_tree(w.scene, w.camera, w.params, 32 * 65 + 32)
    enter = rec[(rec[:, 0] == 2) & (rec[:, 1] == 1)][0]
    leave = rec[(rec[:, 0] == 2) & (rec[:, 1] == 2)][0]
    # on axis: the transmitted ray is undeviated, crosses the diameter and leaves along +z
    _close(enter[5:8], [0, 0, 1])
    assert abs(enter[9] - 2.0) < 3e-3 and enter[10] == 0       # chord length 2 (minus the offsets)
    _close(leave[5:8], [0, 0, 1])
    assert abs(leave[4] - 1.0) < 2e-3                            # leaves at (0,0,+1) plus the offset
    # off axis: two refractions through a sphere deviate the ray by 2 (theta_i - theta_t);
    # exact only without the origin offset, so this FP64 identity uses a tiny one
    w.params.eps = 1e-12
    checked = 0
    for pix in [30 * 65 + 36, 27 * 65 + 33, 34 * 65 + 25, 36 * 65 + 29]:
        rec, _ = oracle.ray_tree(w.scene, w.camera, w.params, pix)
        cam_ray = rec[0]
        if cam_ray[10] != 0:
            continue
        o, d = cam_ray[2:5], cam_ray[5:8]
        x = o + cam_ray[9] * d
        ti = math.acos(min(1.0, -np.dot(d, x)))                    # unit sphere: normal = x
        tt = math.asin(math.sin(ti) / 1.5)
        inside = rec[(rec[:, 0] == 2) & (rec[:, 1] == 1)][0]
        out = rec[(rec[:, 0] == 2) & (rec[:, 1] == 2)][0]
        assert abs(math.acos(np.clip(-np.dot(inside[5:8], x), -1, 1)) - tt) < 1e-9  # Snell: angle to -N
        dev = math.acos(np.clip(np.dot(d, out[5:8]), -1, 1))
        assert abs(dev - 2 * (ti - tt)) < 1e-9
        checked += 1
    assert checked >= 3


def test_no_total_internal_reflection_after_entering_a_sphere():
    glass = S.material((1, 1, 1), k_a=0.0, k_d=0.0, k_s=0.0, ior=1.5, mtype=S.DIELECTRIC)
    w = S.one_sphere(center=(0.0, 0.0, 0.0), radius=1.0, size=97, mat=glass)
    w.params.max_depth = 2
    hits = 0
    for pix in [y * 97 + x for y in range(38, 59, 2) for x in range(38, 59, 2)]:
        rec, _ = oracle.ray_tree(w.scene, w.camera, w.params, pix)
        if rec[0, 10] != 0:
            continue
        hits += 1
        # every entering ray and every exit of a once-refracted ray transmits: no TIR
        assert ((rec[:, 0] == 2) & (rec[:, 1] == 1)).sum() == 1
        assert ((rec[:, 0] == 2) & (rec[:, 1] == 2)).sum() == 1
    assert hits > 30


def test_depth_zero_is_local_only_and_depth_counts():
    w = S.config0()
    w.params.max_depth = 0
    pix = S.pixel_subset(w.camera, 400, 3)
    out = oracle.render(w.scene, w.camera, w.params, pix)
    assert (out["counts"][:, 0, 0] == 1).all()
    # counts: one shadow query per light when N.L > 0 and the term is positive; here <= 1 light
    assert out["counts"][:, 0, 1].max() <= 1
    w.params.max_depth = 3
    out3 = oracle.render(w.scene, w.camera, w.params, pix)
    miss = out["ids"][:, 0] < 0
    _close(out["rgb"][miss], out3["rgb"][miss], atol=0)          # misses do not recurse
    assert (out3["counts"][:, 1, 0] == (~miss)).all()              # each hit (k_r = 0.3) spawns one reflection


def test_config0_is_mostly_robust():
    w = S.config0()
    out = oracle.render(w.scene, w.camera, w.params)
    assert (out["margin"] > 1e-4).mean() >= 0.99
    assert 0.3 < (out["ids"][:, 0] >= 0).mean() < 0.8


# ---------------------------------------------------------------- learned form: the cut-off at a depth

def test_cut_off_render_plus_exact_depth2_radiance_is_the_full_render():
    """Whitted radiance is linear in what the depth-2 rays return: the full image equals the image cut off at
    depth 2 plus, for every depth-2 hit, its path weight times the radiance traced from there.  Pins the
    cut-off's depth, its weights and its background handling (a miss at depth 2 still returns bg) against
    the plain recursion and the per-ray radiance entry."""
    w = S.random_tiny(11, size=40, depth=4)
    w.camera.height = 37
    full = oracle.render(w.scene, w.camera, w.params)
    cut = oracle.render_cache(w.scene, w.camera, w.params, 2)
    rec = cut["records"]
    assert len(rec) > 50
    x, v, wt = rec[:, 1:4], rec[:, 7:10], rec[:, 10:13]
    d = -v
    L, m = oracle.radiance(w.scene, w.params, x - 1e-2 * d, d, 2)      # restart just before each depth-2 hit
    idx = rec[:, 0].astype(int)
    recon = cut["rgb"].copy()
    np.add.at(recon, idx, wt * L)
    ok = (full["margin"] > 1e-4) & (cut["margin"] > 1e-4)
    bad = np.zeros(len(ok), bool)
    bad[idx[m <= 1e-4]] = True
    ok &= ~bad
    assert ok.mean() > 0.9
    _close(recon[ok], full["rgb"][ok], atol=1e-9)
    # the cut-off really removes something on the pixels with depth-2 hits, and nothing elsewhere
    touched = np.zeros(len(ok), bool)
    touched[idx] = True
    assert (np.abs(full["rgb"] - cut["rgb"]).max(axis=1)[ok & touched] > 1e-6).mean() > 0.5
    _close(cut["rgb"][ok & ~touched & (full["counts"][:, 2, 0] == 0)],
           full["rgb"][ok & ~touched & (full["counts"][:, 2, 0] == 0)], atol=1e-12)


def test_cut_off_below_the_maximum_depth_changes_nothing():
    w = S.random_tiny(5, size=24, depth=3)
    full = oracle.render(w.scene, w.camera, w.params)
    cut = oracle.render_cache(w.scene, w.camera, w.params, 4)
    assert len(cut["records"]) == 0
    _close(cut["rgb"], full["rgb"], atol=0)


def test_per_ray_radiance_of_camera_rays_is_the_pixel():
    w = S.config0()
    pix = S.pixel_subset(w.camera, 300, 4)
    out = oracle.render(w.scene, w.camera, w.params, pix)
    o, d = oracle.camera_rays(w.camera, w.params, pix)
    L, m = oracle.radiance(w.scene, w.params, o, d, 0)
    _close(L, out["rgb"], atol=0)


# ---------------------------------------------------------------- area lights sampled once per pass (Section V)

def _disk_light_scene(D=4.0, R=2.0, a=2.0, r=0.5):
    mats = np.stack([S.material((1.0, 1.0, 1.0), k_a=0.0, k_d=1.0, k_s=0.0, k_r=0.0),
                     S.material((0.5, 0.5, 0.5), k_a=0.0, k_d=1.0, k_s=0.0, k_r=0.0)])
    light = [0.0, D, 0.0, 1.0, 1.0, 1.0, S.DISK, R, 0.0, 0.0, 0.0, 0.0, R]
    return S.make_scene(spheres=[[0.0, a, 0.0, r]], sphere_mat=[1], planes=[[0.0, 1.0, 0.0, 0.0]], plane_mat=[0],
                        materials=mats, lights=[light])


def test_disk_light_shadow_of_a_sphere_converges_to_the_area_integral():
    """A Lambert point under a disk light of radius R at height D, with a sphere of radius r at height a on the
    axis between them: a light point at distance rho from the axis is blocked iff rho < (D - e) tan(asin(r /
    (a - e))) (e: the origin offset of the shadow ray), and it contributes N.L = D / sqrt(D^2 + rho^2).  For
    uniform sampling of the disk the pass average converges to
    (2 D / R^2) (sqrt(D^2 + R^2) - sqrt(D^2 + rho0^2))."""
    D, R, a, r = 4.0, 2.0, 2.0, 0.5
    sc = _disk_light_scene(D, R, a, r)
    cam = S.Camera((6.0, 2.0, 0.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 1, 1)
    K = 4095                                    # not a square: every sample goes through the pixel centre
    p = S.Params(spp=K, max_depth=0, jitter=0, seed=11)
    out = oracle.render(sc, cam, p)
    assert (out["ids"][0] == 1).all()          # the plane (id = 1 sphere + 0) at the origin
    e = 1e-3
    rho0 = (D - e) * math.tan(math.asin(r / (a - e)))
    expect = 2.0 * D / R ** 2 * (math.sqrt(D * D + R * R) - math.sqrt(D * D + rho0 * rho0))
    vals = out["rgb_s"][0, :, 0]
    sem = vals.std() / math.sqrt(K)
    assert abs(vals.mean() - expect) < 4.0 * sem, (vals.mean(), expect, sem)
    # the blocked fraction is the area fraction of the inner disk, (rho0 / R)^2
    assert abs((vals == 0.0).mean() - (rho0 / R) ** 2) < 4.0 * math.sqrt(0.25 / K)
    # a point light at the disk centre: fully blocked
    sc0 = _disk_light_scene(D, R, a, r)
    sc0.lights[0, 6] = S.POINT
    assert oracle.render(sc0, cam, S.Params(spp=1, max_depth=0, jitter=0))["rgb"][0, 0] == 0.0


def test_light_points_cover_their_shapes_uniformly():
    n = 20000
    disk = np.array([1.0, 2.0, 3.0, 1, 1, 1, S.DISK, 0.0, 2.0, 0.0, 0.0, 0.0, 2.0], np.float32)
    quad = np.array([1.0, 2.0, 3.0, 1, 1, 1, S.PARALLELOGRAM, 4.0, 0.0, 0.0, 1.0, 0.0, 3.0], np.float32)
    pd = np.array([oracle.light_point(disk, 7, 3, s, 2) for s in range(n)])
    pq = np.array([oracle.light_point(quad, 7, 3, s, 0) for s in range(n)])
    # disk: in the plane x = 1 around (1, 2, 3), radius 2; P(rho < t) = (t / 2)^2; centred
    assert np.abs(pd[:, 0] - 1.0).max() < 1e-6
    rho = np.hypot(pd[:, 1] - 2.0, pd[:, 2] - 3.0)
    assert rho.max() <= 2.0 + 1e-5
    for t in (0.5, 1.0, 1.5):
        assert abs((rho < t).mean() - (t / 2.0) ** 2) < 4 * math.sqrt(0.25 / n)
    assert np.abs(pd[:, 1:].mean(0) - [2.0, 3.0]).max() < 0.05
    # parallelogram: coordinates (a, b) = ((x - 1 - (z - 3) / 3) / 4, (z - 3) / 3) uniform in [0, 1)^2
    b = (pq[:, 2] - 3.0) / 3.0
    a = (pq[:, 0] - 1.0 - 1.0 * b) / 4.0
    assert a.min() >= -1e-6 and a.max() < 1 + 1e-6 and b.min() >= -1e-6 and b.max() < 1 + 1e-6
    assert np.abs(pq[:, 1] - 2.0).max() < 1e-6
    for q in (0.25, 0.5, 0.75):
        assert abs((a < q).mean() - q) < 4 * math.sqrt(0.25 / n) and abs((b < q).mean() - q) < 4 * math.sqrt(0.25 / n)
    # different lights, frames and samples draw different points; a point light is its position
    assert not np.allclose(oracle.light_point(disk, 7, 3, 0, 0), oracle.light_point(disk, 7, 3, 0, 1))
    assert not np.allclose(oracle.light_point(disk, 7, 3, 0, 0), oracle.light_point(disk, 7, 4, 0, 0))
    pt = disk.copy()
    pt[6] = S.POINT
    assert (oracle.light_point(pt, 7, 3, 5, 0) == [1.0, 2.0, 3.0]).all()
