// Host-side exercise of the library's CPU code (scene validation, binned-SAH
// BVH build, the five node layouts, packing, the host FP32 traversal) for a
// build with AddressSanitizer and UndefinedBehaviorSanitizer.  No GPU call is
// made.  Exit status 0 when every check passes; a sanitizer report aborts.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "mirt.h"

static int failures = 0;
#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

struct Arrays {
    std::vector<float> spheres, tris, planes;
    std::vector<int32_t> smat, tmat, pmat;
    std::vector<rt_material> mats;
    std::vector<rt_light> lights;
    rt_scene_desc desc() const {
        rt_scene_desc d{};
        d.spheres = spheres.empty() ? nullptr : spheres.data();
        d.n_spheres = (int64_t)smat.size();
        d.sphere_mat = smat.empty() ? nullptr : smat.data();
        d.tris = tris.empty() ? nullptr : tris.data();
        d.n_tris = (int64_t)tmat.size();
        d.tri_mat = tmat.empty() ? nullptr : tmat.data();
        d.planes = planes.empty() ? nullptr : planes.data();
        d.n_planes = (int64_t)pmat.size();
        d.plane_mat = pmat.empty() ? nullptr : pmat.data();
        d.materials = mats.data();
        d.n_materials = (int32_t)mats.size();
        d.lights = lights.data();
        d.n_lights = (int32_t)lights.size();
        return d;
    }
};

static Arrays random_scene(unsigned seed, int ns, int nt, int np) {
    std::mt19937 g(seed);
    std::uniform_real_distribution<float> u(-5.0f, 5.0f), r(0.1f, 1.0f), s(-0.8f, 0.8f);
    Arrays a;
    rt_material m{};
    m.albedo[0] = m.albedo[1] = m.albedo[2] = 0.5f;
    m.k_a = 0.1f; m.k_d = 1.0f; m.k_s = 0.5f; m.shininess = 32.0f; m.k_r = 0.2f; m.ior = 1.5f;
    for (int t = 0; t < 3; ++t) { m.type = t; a.mats.push_back(m); }
    rt_light l{};
    l.pos[1] = 10.0f; l.intensity[0] = l.intensity[1] = l.intensity[2] = 1.0f;
    a.lights.push_back(l);
    for (int i = 0; i < ns; ++i) {
        a.spheres.insert(a.spheres.end(), {u(g), u(g), u(g), r(g)});
        a.smat.push_back(i % 3);
    }
    for (int i = 0; i < nt; ++i) {
        const float cx = u(g), cy = u(g), cz = u(g);
        for (int v = 0; v < 3; ++v) a.tris.insert(a.tris.end(), {cx + s(g), cy + s(g), cz + s(g)});
        a.tmat.push_back(i % 3);
    }
    if (nt > 4) {   // a zero-area triangle and two identical ones
        for (int k = 0; k < 9; ++k) a.tris[9 + k] = (float)(k % 3);
        for (int k = 0; k < 9; ++k) a.tris[18 + k] = a.tris[27 + k];
    }
    for (int i = 0; i < np; ++i) {
        a.planes.insert(a.planes.end(), {0.0f, 1.0f, 0.0f, -6.0f - (float)i});
        a.pmat.push_back(0);
    }
    return a;
}

static void traverse_all_layouts(const Arrays& a, int leaf_max, int bins, unsigned seed) {
    rt_build_opts o{};
    o.leaf_max = leaf_max;
    o.sah_bins = bins;
    rt_scene* sc = nullptr;
    const rt_scene_desc d = a.desc();
    if (rt_build_scene(&d, &o, &sc) != RT_OK) {
        std::fprintf(stderr, "build failed: %s\n", rt_last_error());
        ++failures;
        return;
    }
    const int n = 4000;
    std::mt19937 g(seed);
    std::uniform_real_distribution<float> u(-7.0f, 7.0f), dn(-1.0f, 1.0f), tm(0.5f, 12.0f);
    std::vector<float> rays(8 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        float dx = dn(g), dy = dn(g), dz = dn(g);
        const float len = std::sqrt(dx * dx + dy * dy + dz * dz) + 1e-6f;
        float* R = &rays[8 * (size_t)i];
        R[0] = u(g); R[1] = u(g); R[2] = u(g);
        R[3] = dx / len; R[4] = dy / len; R[5] = dz / len;
        R[6] = 0.0f; R[7] = (i % 2) ? tm(g) : 0.0f;
    }
    std::vector<float> t0(n), t(n);
    std::vector<int32_t> id0(n), id(n), occ0(n), occ(n);
    std::vector<uint32_t> work(3 * (size_t)n);
    for (int layout = RT_LAYOUT_DFS; layout <= RT_LAYOUT_BVH4Q; ++layout) {
        CHECK(rt_scene_set_layout(sc, layout) == RT_OK);
        rt_scene_info info{};
        CHECK(rt_scene_get_info(sc, &info) == RT_OK && info.node_layout == layout);
        CHECK(rt_scene_device_bytes(sc) > 0);
        const bool first = layout == RT_LAYOUT_DFS;
        CHECK(rt_host_trace(sc, rays.data(), n, 0, first ? t0.data() : t.data(), first ? id0.data() : id.data(),
                            work.data(), 3) == RT_OK);
        CHECK(rt_host_trace(sc, rays.data(), n, 1, t.data(), first ? occ0.data() : occ.data(), nullptr, 2) == RT_OK);
        if (!first) {
            int diff = 0;
            for (int i = 0; i < n; ++i) diff += (id[i] != id0[i]) + ((occ[i] >= 0) != (occ0[i] >= 0));
            CHECK(diff == 0);   // every layout answers every query the same way
        }
    }
    rt_destroy_scene(sc);
}

int main() {
    // scenes of every kind: spheres only, triangles only, mixed with planes, one primitive, planes only
    const int cfg[][3] = {{40, 0, 0}, {0, 600, 0}, {25, 400, 2}, {1, 0, 0}, {0, 1, 1}, {0, 0, 3}, {3, 5000, 1}};
    unsigned seed = 1;
    for (const auto& c : cfg)
        for (int leaf : {1, 4, 15})
            traverse_all_layouts(random_scene(seed++, c[0], c[1], c[2]), leaf, leaf == 4 ? 0 : 16, seed);
    // validation errors leave nothing behind
    Arrays bad = random_scene(99, 4, 4, 1);
    bad.spheres[3] = -1.0f;
    rt_scene* sc = nullptr;
    rt_scene_desc d = bad.desc();
    CHECK(rt_build_scene(&d, nullptr, &sc) == RT_ERR_INVALID_ARG && sc == nullptr);
    bad = random_scene(98, 4, 4, 1);
    bad.tris[5] = NAN;
    d = bad.desc();
    CHECK(rt_build_scene(&d, nullptr, &sc) == RT_ERR_INVALID_ARG);
    bad = random_scene(97, 4, 4, 1);
    bad.tmat[2] = 7;
    d = bad.desc();
    CHECK(rt_build_scene(&d, nullptr, &sc) == RT_ERR_INVALID_ARG);
    bad = random_scene(96, 4, 4, 1);
    bad.planes[0] = 2.0f;
    d = bad.desc();
    CHECK(rt_build_scene(&d, nullptr, &sc) == RT_ERR_INVALID_ARG);
    // a depth limit that the tree exceeds
    Arrays deep = random_scene(95, 0, 3000, 0);
    rt_build_opts o{};
    o.leaf_max = 1;
    o.max_depth = 3;
    d = deep.desc();
    CHECK(rt_build_scene(&d, &o, &sc) == RT_ERR_BVH_DEPTH);
    CHECK(rt_build_scene(nullptr, nullptr, &sc) != RT_OK);
    std::printf("host sanitizer driver: %d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
