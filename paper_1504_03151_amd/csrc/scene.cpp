// scene.cpp -- scene validation, binned-SAH BVH build, packing, upload and the
// host FP32 traversal behind the C ABI (include/mirt.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "bvh_quant.h"
#include "mirt_internal.h"

namespace mirt {

static thread_local std::string g_last_error;
static std::atomic<uint64_t> g_scene_uid{1};

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

struct Box {
    float lo[3], hi[3];
    void reset() {
        for (int k = 0; k < 3; ++k) {
            lo[k] = INFINITY;
            hi[k] = -INFINITY;
        }
    }
    void grow(const Box& b) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], b.lo[k]);
            hi[k] = std::max(hi[k], b.hi[k]);
        }
    }
    void grow(const float* p) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], p[k]);
            hi[k] = std::max(hi[k], p[k]);
        }
    }
    bool empty() const { return lo[0] > hi[0]; }
    double area() const {
        if (empty()) return 0.0;
        const double x = (double)hi[0] - lo[0], y = (double)hi[1] - lo[1], z = (double)hi[2] - lo[2];
        return 2.0 * (x * y + y * z + z * x);
    }
};

struct Ref {
    Box box;
    float c[3];
    int32_t prim;  // combined index: sphere i -> i, triangle j -> ns + j
};

struct Builder {
    std::vector<Ref>& refs;
    std::vector<Node>& nodes;
    int bins, leaf_max, max_depth;
    float pad;
    int depth_reached = 0;
    int64_t leaves = 0;
    double sah_sum = 0.0;   // sum of area-weighted costs (normalised later)
    bool too_deep = false;

    Builder(std::vector<Ref>& r, std::vector<Node>& n, int b, int lm, int md, float p)
        : refs(r), nodes(n), bins(b), leaf_max(lm), max_depth(md), pad(p) {}

    Box padded(Box b) const {
        if (b.empty()) return b;
        for (int k = 0; k < 3; ++k) {
            b.lo[k] -= pad;
            b.hi[k] += pad;
        }
        return b;
    }

    int32_t make_leaf(int begin, int end, const Box& box) {
        leaves++;
        sah_sum += box.area() * (end - begin);
        return leaf_ref(begin, end - begin);
    }

    // Build the subtree over refs[begin, end); returns its child reference and box.
    int32_t build(int begin, int end, int depth, Box& box_out, bool force_node) {
        const int n = end - begin;
        Box box, cbox;
        box.reset();
        cbox.reset();
        for (int i = begin; i < end; ++i) {
            box.grow(refs[i].box);
            cbox.grow(refs[i].c);
        }
        box_out = box;
        depth_reached = std::max(depth_reached, depth);
        if (!force_node) {
            if (n <= 1 || (depth >= max_depth && n <= kLeafMaxCount)) return make_leaf(begin, end, box);
            if (depth >= max_depth) {
                too_deep = true;
                return make_leaf(begin, begin + kLeafMaxCount, box);
            }
        }
        // binned SAH over centroids
        int best_axis = -1, best_bin = -1;
        double best_cost = INFINITY;
        std::vector<Box> bb(bins);
        std::vector<int> bc(bins);
        std::vector<double> rarea(bins);
        std::vector<int> rcount(bins);
        for (int ax = 0; ax < 3; ++ax) {
            const float lo = cbox.lo[ax], hi = cbox.hi[ax];
            if (!(hi > lo)) continue;
            const float scale = bins / (hi - lo);
            for (int b = 0; b < bins; ++b) {
                bb[b].reset();
                bc[b] = 0;
            }
            for (int i = begin; i < end; ++i) {
                int b = (int)((refs[i].c[ax] - lo) * scale);
                b = std::min(std::max(b, 0), bins - 1);
                bb[b].grow(refs[i].box);
                bc[b]++;
            }
            Box acc;
            acc.reset();
            int cnt = 0;
            for (int b = bins - 1; b > 0; --b) {
                acc.grow(bb[b]);
                cnt += bc[b];
                rarea[b] = acc.area();
                rcount[b] = cnt;
            }
            acc.reset();
            cnt = 0;
            for (int b = 0; b < bins - 1; ++b) {
                acc.grow(bb[b]);
                cnt += bc[b];
                const int rc = rcount[b + 1];
                if (cnt == 0 || rc == 0) continue;
                const double cost = acc.area() * cnt + rarea[b + 1] * rc;
                if (cost < best_cost) {
                    best_cost = cost;
                    best_axis = ax;
                    best_bin = b;
                }
            }
        }
        const double parea = std::max(box.area(), 1e-30);
        const double leaf_cost = (double)n;                     // C_isect = 1 per primitive
        const double split_cost = 1.0 + best_cost / parea;      // C_trav = 1
        if (!force_node && n <= leaf_max && (best_axis < 0 || leaf_cost <= split_cost))
            return make_leaf(begin, end, box);
        int mid;
        if (best_axis < 0) {
            // coincident centroids: any partition is as good; keep leaves small
            if (!force_node && n <= kLeafMaxCount) return make_leaf(begin, end, box);
            mid = begin + n / 2;
        } else {
            const float lo = cbox.lo[best_axis], hi = cbox.hi[best_axis];
            const float scale = bins / (hi - lo);
            auto it = std::partition(refs.begin() + begin, refs.begin() + end, [&](const Ref& r) {
                int b = (int)((r.c[best_axis] - lo) * scale);
                b = std::min(std::max(b, 0), bins - 1);
                return b <= best_bin;
            });
            mid = (int)(it - refs.begin());
            if (mid == begin || mid == end) mid = begin + n / 2;
        }
        if (n == 1) {
            // forced inner node over a single primitive: leaf on the left, empty right
            const int32_t idx = (int32_t)nodes.size();
            nodes.emplace_back();
            Box lb = padded(box);
            Node& nd = nodes[idx];
            nd.a = make_float4(lb.lo[0], lb.hi[0], lb.lo[1], lb.hi[1]);
            nd.b = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
            nd.c = make_float4(lb.lo[2], lb.hi[2], INFINITY, -INFINITY);
            nd.d = make_int4(make_leaf(begin, end, box), leaf_ref(0, 0), 0, 0);
            return idx;
        }
        const int32_t idx = (int32_t)nodes.size();
        nodes.emplace_back();
        sah_sum += box.area();
        Box lb, rb;
        const int32_t cl = build(begin, mid, depth + 1, lb, false);
        const int32_t cr = build(mid, end, depth + 1, rb, false);
        lb = padded(lb);
        rb = padded(rb);
        Node& nd = nodes[idx];
        nd.a = make_float4(lb.lo[0], lb.hi[0], lb.lo[1], lb.hi[1]);
        nd.b = make_float4(rb.lo[0], rb.hi[0], rb.lo[1], rb.hi[1]);
        nd.c = make_float4(lb.lo[2], lb.hi[2], rb.lo[2], rb.hi[2]);
        nd.d = make_int4(cl, cr, 0, 0);
        return idx;
    }
};

// Node order in memory.  Every layout keeps the root at index 0 and only
// renumbers inner-node references, so traversal visits the same nodes in the
// same order and returns the same hits whatever the layout.
constexpr size_t kTreeletNodes = 7;   // three levels of a binary subtree

std::vector<int32_t> layout_order(const std::vector<Node>& nodes, int layout) {
    std::vector<int32_t> order;
    order.reserve(nodes.size());
    if (nodes.empty()) return order;
    if (layout == RT_LAYOUT_BFS) {
        order.push_back(0);
        for (size_t h = 0; h < order.size(); ++h) {
            const int4 d = nodes[order[h]].d;
            if (d.x >= 0) order.push_back(d.x);
            if (d.y >= 0) order.push_back(d.y);
        }
    } else if (layout == RT_LAYOUT_TREELET) {
        std::vector<int32_t> roots{0}, blk, below;
        while (!roots.empty()) {
            const int32_t r = roots.back();
            roots.pop_back();
            blk.assign(1, r);
            below.clear();
            for (size_t h = 0; h < blk.size(); ++h) {
                const int4 d = nodes[blk[h]].d;
                for (int32_t c : {d.x, d.y}) {
                    if (c < 0) continue;
                    if (blk.size() < kTreeletNodes) blk.push_back(c);
                    else below.push_back(c);
                }
            }
            order.insert(order.end(), blk.begin(), blk.end());
            roots.insert(roots.end(), below.rbegin(), below.rend());   // left-most block next
        }
    } else {   // depth-first pre-order, left subtree first
        std::vector<int32_t> st{0};
        while (!st.empty()) {
            const int32_t i = st.back();
            st.pop_back();
            order.push_back(i);
            const int4 d = nodes[i].d;
            if (d.y >= 0) st.push_back(d.y);
            if (d.x >= 0) st.push_back(d.x);
        }
    }
    return order;
}

void apply_layout(Node* nodes, int64_t n, int layout) {
    std::vector<Node> old(nodes, nodes + n);
    const std::vector<int32_t> order = layout_order(old, layout);
    if ((int64_t)order.size() != n) throw std::runtime_error("BVH node layout: tree does not reach every node");
    std::vector<int32_t> pos(n);
    for (int64_t k = 0; k < n; ++k) pos[order[k]] = (int32_t)k;
    for (int64_t k = 0; k < n; ++k) {
        Node nd = old[order[k]];
        if (nd.d.x >= 0) nd.d.x = pos[nd.d.x];
        if (nd.d.y >= 0) nd.d.y = pos[nd.d.y];
        nodes[k] = nd;
    }
}

// Four-wide collapse of the binary tree: a four-wide node takes the two
// children of a binary node and keeps opening the inner child with the largest
// box surface until it holds four children or only leaves are left.  Child
// boxes are copied unchanged (already padded); an empty box becomes the
// all-+inf box no slab test accepts.
struct Child4 {
    float lo[3], hi[3];
    int32_t ref;
};

void binary_children(const Node& n, Child4& l, Child4& r) {
    l = Child4{{n.a.x, n.a.z, n.c.x}, {n.a.y, n.a.w, n.c.y}, n.d.x};
    r = Child4{{n.b.x, n.b.z, n.c.z}, {n.b.y, n.b.w, n.c.w}, n.d.y};
}

double child_area(const Child4& c) {
    const double e0 = (double)c.hi[0] - c.lo[0], e1 = (double)c.hi[1] - c.lo[1], e2 = (double)c.hi[2] - c.lo[2];
    if (!(e0 >= 0.0 && e1 >= 0.0 && e2 >= 0.0)) return -1.0;
    return e0 * e1 + e1 * e2 + e2 * e0;
}

int32_t collapse4(const std::vector<Node>& n2, int32_t idx, int depth, std::vector<Node4>& out, int& max_depth) {
    Child4 e[4];
    int k = 2;
    binary_children(n2[idx], e[0], e[1]);
    while (k < 4) {
        int best = -1;
        double ba = -2.0;
        for (int i = 0; i < k; ++i)
            if (e[i].ref >= 0 && child_area(e[i]) > ba) {
                best = i;
                ba = child_area(e[i]);
            }
        if (best < 0) break;
        Child4 l, r;
        binary_children(n2[e[best].ref], l, r);
        e[best] = l;
        e[k++] = r;
    }
    const int32_t me = (int32_t)out.size();
    out.emplace_back();
    max_depth = std::max(max_depth, depth);
    int32_t refs[4];
    for (int i = 0; i < k; ++i) refs[i] = e[i].ref >= 0 ? collapse4(n2, e[i].ref, depth + 1, out, max_depth) : e[i].ref;
    float b[6][4];
    int32_t c[4];
    for (int i = 0; i < 4; ++i) {
        const bool used = i < k && child_area(e[i]) >= 0.0;
        for (int a = 0; a < 3; ++a) {
            b[2 * a][i] = used ? e[i].lo[a] : INFINITY;
            b[2 * a + 1][i] = used ? e[i].hi[a] : INFINITY;
        }
        c[i] = i < k ? refs[i] : leaf_ref(0, 0);
    }
    Node4& o = out[me];
    o.lox = make_float4(b[0][0], b[0][1], b[0][2], b[0][3]);
    o.hix = make_float4(b[1][0], b[1][1], b[1][2], b[1][3]);
    o.loy = make_float4(b[2][0], b[2][1], b[2][2], b[2][3]);
    o.hiy = make_float4(b[3][0], b[3][1], b[3][2], b[3][3]);
    o.loz = make_float4(b[4][0], b[4][1], b[4][2], b[4][3]);
    o.hiz = make_float4(b[5][0], b[5][1], b[5][2], b[5][3]);
    o.child = make_int4(c[0], c[1], c[2], c[3]);
    o.pad = make_int4(0, 0, 0, 0);
    return me;
}

// 8-bit quantization of a four-wide node's child boxes (RT_LAYOUT_BVH4Q): the
// shared quantizer of bvh_quant.h (the device refit uses the same code).
float f4c(const float4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }

bool quantize4(const Node4& n, Node4q& q) {
    float lo[4][3], hi[4][3];
    bool valid[4];
    const float4* L[3] = {&n.lox, &n.loy, &n.loz};
    const float4* H[3] = {&n.hix, &n.hiy, &n.hiz};
    for (int i = 0; i < 4; ++i) {
        for (int a = 0; a < 3; ++a) {
            lo[i][a] = f4c(*L[a], i);
            hi[i][a] = f4c(*H[a], i);
        }
        valid[i] = std::isfinite(lo[i][0]) && std::isfinite(hi[i][0]);
    }
    return quantize_children(lo, hi, valid, n.child, q);
}

// Node section of a layout (bytes), with the node count and the traversal
// stack entries a ray needs in it.  Returns false if that stack would not fit.
bool layout_nodes(const std::vector<Node>& dfs, int layout, int depth2, std::vector<uint8_t>& bytes, int64_t& n_nodes,
                  int& stack_size) {
    if (layout == RT_LAYOUT_BVH4 || layout == RT_LAYOUT_BVH4Q) {
        std::vector<Node4> n4;
        n4.reserve(dfs.size() / 2 + 1);
        int d4 = 0;
        collapse4(dfs, 0, 0, n4, d4);
        // at most three siblings pushed per level on the way down, plus the
        // end marker and the pushes of the deepest node
        stack_size = 3 * d4 + 5;
        if (stack_size > kMaxStack) return false;
        n_nodes = (int64_t)n4.size();
        if (layout == RT_LAYOUT_BVH4) {
            bytes.resize(n4.size() * sizeof(Node4));
            std::memcpy(bytes.data(), n4.data(), bytes.size());
            return true;
        }
        std::vector<Node4q> nq(n4.size());
        for (size_t i = 0; i < n4.size(); ++i)
            if (!quantize4(n4[i], nq[i])) return false;
        bytes.resize(nq.size() * sizeof(Node4q));
        std::memcpy(bytes.data(), nq.data(), bytes.size());
        return true;
    }
    std::vector<Node> v = dfs;
    if (layout != RT_LAYOUT_DFS) apply_layout(v.data(), (int64_t)v.size(), layout);
    stack_size = depth2 + 3;
    bytes.resize(v.size() * sizeof(Node));
    std::memcpy(bytes.data(), v.data(), bytes.size());
    n_nodes = (int64_t)v.size();
    return true;
}

bool finite3(const float* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

// Child references of node i of a node section in the given layout (4 slots; binary nodes fill 2).
int node_children(const uint8_t* nodes, int layout, int64_t i, int32_t (&ch)[4]) {
    if (layout == RT_LAYOUT_BVH4) {
        const int4 c = reinterpret_cast<const Node4*>(nodes)[i].child;
        ch[0] = c.x, ch[1] = c.y, ch[2] = c.z, ch[3] = c.w;
        return 4;
    }
    if (layout == RT_LAYOUT_BVH4Q) {
        const Node4q& q = reinterpret_cast<const Node4q*>(nodes)[i];
        ch[0] = (int32_t)q.qb.z, ch[1] = (int32_t)q.qb.w, ch[2] = q.qc.x, ch[3] = q.qc.y;
        return 4;
    }
    const int4 d = reinterpret_cast<const Node*>(nodes)[i].d;
    ch[0] = d.x, ch[1] = d.y;
    return 2;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Refit order: node indices grouped by depth below the root, deepest level
// first, so that a level's children were refit by an earlier level.
void refit_schedule(SceneHost& h) {
    const int64_t n = h.n_nodes;
    const uint8_t* nb = h.blob.data() + h.off_nodes;
    std::vector<int32_t> depth(n, -1), bfs;
    bfs.reserve(n);
    bfs.push_back(0);
    depth[0] = 0;
    int maxd = 0;
    for (size_t k = 0; k < bfs.size(); ++k) {
        int32_t ch[4];
        const int nc = node_children(nb, h.layout, bfs[k], ch);
        for (int c = 0; c < nc; ++c)
            if (ch[c] >= 0) {
                if (ch[c] >= n || depth[ch[c]] >= 0) throw std::runtime_error("refit schedule: malformed tree");
                depth[ch[c]] = depth[bfs[k]] + 1;
                maxd = std::max(maxd, depth[ch[c]]);
                bfs.push_back(ch[c]);
            }
    }
    if ((int64_t)bfs.size() != n) throw std::runtime_error("refit schedule: tree does not reach every node");
    h.refit_levels.assign(maxd + 2, 0);
    for (int64_t i = 0; i < n; ++i) h.refit_levels[maxd - depth[i] + 1]++;
    for (int l = 0; l <= maxd; ++l) h.refit_levels[l + 1] += h.refit_levels[l];
    std::vector<int64_t> next(h.refit_levels.begin(), h.refit_levels.end() - 1);
    h.blob.resize(h.off_refit + align256(4 * (size_t)n));
    int32_t* order = reinterpret_cast<int32_t*>(h.blob.data() + h.off_refit);
    for (int64_t i = 0; i < n; ++i) order[next[maxd - depth[i]]++] = (int32_t)i;
}

}  // namespace mirt

using namespace mirt;

extern "C" {

const char* rt_last_error(void) { return g_last_error.c_str(); }
const char* rt_version(void) { return "mirt 0.1 (gfx950)"; }

rt_status rt_build_scene(const rt_scene_desc* desc, const rt_build_opts* opts, rt_scene** out) {
    try {
        if (!desc || !out) {
            set_error("rt_build_scene: NULL argument");
            return RT_ERR_INVALID_ARG;
        }
        *out = nullptr;
        const int64_t ns = desc->n_spheres, nt = desc->n_tris, np = desc->n_planes;
        const int nm = desc->n_materials, nl = desc->n_lights;
        if (ns < 0 || nt < 0 || np < 0 || nm < 0 || nl < 0) {
            set_error("rt_build_scene: negative count");
            return RT_ERR_INVALID_ARG;
        }
        if ((ns && (!desc->spheres || !desc->sphere_mat)) || (nt && (!desc->tris || !desc->tri_mat)) ||
            (np && (!desc->planes || !desc->plane_mat)) || (nm && !desc->materials) || (nl && !desc->lights)) {
            set_error("rt_build_scene: NULL array with a non-zero count");
            return RT_ERR_INVALID_ARG;
        }
        if (ns + nt >= ((int64_t)1 << 27) || np > 4096 || nl > 1024) {
            set_error("rt_build_scene: too many primitives (< 2^27 spheres + triangles, <= 4096 planes, "
                      "<= 1024 lights)");
            return RT_ERR_UNSUPPORTED;
        }
        if (ns + nt + np > 0 && nm == 0) {
            set_error("rt_build_scene: primitives need at least one material");
            return RT_ERR_INVALID_ARG;
        }
        for (int m = 0; m < nm; ++m) {
            const rt_material& M = desc->materials[m];
            const float v[9] = {M.albedo[0], M.albedo[1], M.albedo[2], M.k_a, M.k_d, M.k_s, M.shininess, M.k_r,
                                M.ior};
            for (float f : v)
                if (!std::isfinite(f)) {
                    set_error("rt_build_scene: non-finite material " + std::to_string(m));
                    return RT_ERR_INVALID_ARG;
                }
            if (M.type < RT_MAT_PHONG || M.type > RT_MAT_DIELECTRIC || M.shininess < 0.0f ||
                (M.type == RT_MAT_DIELECTRIC && !(M.ior > 0.0f))) {
                set_error("rt_build_scene: invalid material " + std::to_string(m));
                return RT_ERR_INVALID_ARG;
            }
        }
        for (int l = 0; l < nl; ++l) {
            const rt_light& L = desc->lights[l];
            if (!finite3(L.pos) || !finite3(L.intensity) || L.shape < RT_LIGHT_POINT || L.shape > RT_LIGHT_DISK ||
                (L.shape != RT_LIGHT_POINT && (!finite3(L.u) || !finite3(L.v)))) {
                set_error("rt_build_scene: invalid light " + std::to_string(l) + " (non-finite or unknown shape)");
                return RT_ERR_INVALID_ARG;
            }
        }
        float scale = 1.0f;
        for (int64_t i = 0; i < ns; ++i) {
            const float* s = desc->spheres + 4 * i;
            if (!finite3(s) || !std::isfinite(s[3]) || !(s[3] > 0.0f)) {
                set_error("rt_build_scene: invalid sphere " + std::to_string(i) + " (non-finite or r <= 0)");
                return RT_ERR_INVALID_ARG;
            }
            if (desc->sphere_mat[i] < 0 || desc->sphere_mat[i] >= nm) {
                set_error("rt_build_scene: sphere " + std::to_string(i) + " material out of range");
                return RT_ERR_INVALID_ARG;
            }
            for (int k = 0; k < 3; ++k) scale = std::max(scale, std::fabs(s[k]) + s[3]);
        }
        for (int64_t i = 0; i < nt; ++i) {
            const float* t = desc->tris + 9 * i;
            if (!finite3(t) || !finite3(t + 3) || !finite3(t + 6)) {
                set_error("rt_build_scene: non-finite triangle " + std::to_string(i));
                return RT_ERR_INVALID_ARG;
            }
            if (desc->tri_mat[i] < 0 || desc->tri_mat[i] >= nm) {
                set_error("rt_build_scene: triangle " + std::to_string(i) + " material out of range");
                return RT_ERR_INVALID_ARG;
            }
            for (int k = 0; k < 9; ++k) scale = std::max(scale, std::fabs(t[k]));
        }
        for (int64_t i = 0; i < np; ++i) {
            const float* p = desc->planes + 4 * i;
            const double nn = (double)p[0] * p[0] + (double)p[1] * p[1] + (double)p[2] * p[2];
            if (!finite3(p) || !std::isfinite(p[3]) || std::fabs(std::sqrt(nn) - 1.0) > 1e-3) {
                set_error("rt_build_scene: invalid plane " + std::to_string(i) + " (needs finite n, |n| = 1)");
                return RT_ERR_INVALID_ARG;
            }
            if (desc->plane_mat[i] < 0 || desc->plane_mat[i] >= nm) {
                set_error("rt_build_scene: plane " + std::to_string(i) + " material out of range");
                return RT_ERR_INVALID_ARG;
            }
        }
        rt_build_opts o{};
        if (opts) o = *opts;
        const int leaf_max = o.leaf_max > 0 ? std::min(o.leaf_max, kLeafMaxCount) : 4;
        const int bins = o.sah_bins > 1 ? std::min(o.sah_bins, 256) : 32;
        const int max_depth = o.max_depth > 0 ? std::min(o.max_depth, 61) : 60;
        if (o.node_layout < RT_LAYOUT_DFS || o.node_layout > RT_LAYOUT_BVH4Q) {
            set_error("rt_build_scene: node_layout must be one of RT_LAYOUT_DFS, _BFS, _TREELET, _BVH4, _BVH4Q");
            return RT_ERR_INVALID_ARG;
        }

        const auto t0 = std::chrono::steady_clock::now();
        std::vector<Ref> refs((size_t)(ns + nt));
        for (int64_t i = 0; i < ns; ++i) {
            const float* s = desc->spheres + 4 * i;
            Ref& r = refs[i];
            for (int k = 0; k < 3; ++k) {
                r.box.lo[k] = s[k] - s[3];
                r.box.hi[k] = s[k] + s[3];
                r.c[k] = s[k];
            }
            r.prim = (int32_t)i;
        }
        for (int64_t j = 0; j < nt; ++j) {
            const float* t = desc->tris + 9 * j;
            Ref& r = refs[ns + j];
            r.box.reset();
            for (int v = 0; v < 3; ++v) r.box.grow(t + 3 * v);
            for (int k = 0; k < 3; ++k) r.c[k] = (float)(((double)t[k] + t[3 + k] + t[6 + k]) / 3.0);
            r.prim = (int32_t)(ns + j);
        }
        std::vector<Node> nodes;
        nodes.reserve((size_t)std::max<int64_t>(1, (ns + nt) / 2 + 1));
        // outward box padding: FP32 slab tests of rays with origins and hits within
        // the scene's magnitude stay conservative
        const float pad = scale * 0x1p-19f;
        Builder B(refs, nodes, bins, leaf_max, max_depth, pad);
        Box root;
        if (ns + nt == 0) {
            Node nd;
            nd.a = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
            nd.b = nd.a;
            nd.c = nd.a;
            nd.d = make_int4(leaf_ref(0, 0), leaf_ref(0, 0), 0, 0);
            nodes.push_back(nd);
            root.reset();
        } else {
            B.build(0, (int)(ns + nt), 0, root, true);
        }
        if (B.too_deep) {
            set_error("rt_build_scene: BVH deeper than max_depth " + std::to_string(max_depth));
            return RT_ERR_BVH_DEPTH;
        }
        std::vector<uint8_t> node_bytes;
        int64_t n_nodes = 0;
        int stack_size = 0;
        if (!layout_nodes(nodes, o.node_layout, B.depth_reached, node_bytes, n_nodes, stack_size)) {
            set_error("rt_build_scene: four-wide traversal stack would exceed " + std::to_string(kMaxStack) + " entries");
            return RT_ERR_BVH_DEPTH;
        }
        const auto t1 = std::chrono::steady_clock::now();

        SceneHost h;
        h.n_spheres = (int)ns;
        h.n_tris = (int)nt;
        h.n_planes = (int)np;
        h.n_lights = nl;
        h.n_materials = nm;
        h.n_nodes = n_nodes;
        h.depth = B.depth_reached;
        h.stack_size = stack_size;
        h.layout = o.node_layout;
        for (int l = 0; l < nl; ++l) h.area_lights = h.area_lights || desc->lights[l].shape != RT_LIGHT_POINT;
        h.scale = scale;
        const int64_t nb = ns + nt;
        size_t off = 0;
        h.off_nodes = off;
        off = align256(off + node_bytes.size());
        h.off_prims = off;
        off = align256(off + 48 * (size_t)std::max<int64_t>(nb, 1));
        h.off_normals = off;
        off = align256(off + 16 * (size_t)std::max<int64_t>(nb, 1));
        h.off_planes = off;
        off = align256(off + 16 * (size_t)std::max<int64_t>(np, 1));
        h.off_plane_mat = off;
        off = align256(off + 4 * (size_t)std::max<int64_t>(np, 1));
        h.off_mats = off;
        off = align256(off + sizeof(DevMaterial) * (size_t)std::max(nm, 1));
        h.off_lights = off;
        off = align256(off + sizeof(DevLight) * (size_t)std::max(nl, 1));
        h.off_refit = off;
        off = align256(off + 4 * (size_t)n_nodes);
        h.blob.assign(off, 0);
        uint8_t* base = h.blob.data();
        std::memcpy(base + h.off_nodes, node_bytes.data(), node_bytes.size());
        float4* prims = reinterpret_cast<float4*>(base + h.off_prims);
        float4* normals = reinterpret_cast<float4*>(base + h.off_normals);
        for (int64_t i = 0; i < nb; ++i) {
            const int32_t p = refs[i].prim;
            if (p < ns) {
                const float* s = desc->spheres + 4 * p;
                prims[3 * i] = make_float4(s[0], s[1], s[2], as_float_i(p));
                prims[3 * i + 1] = make_float4(s[3], s[3] * s[3], 1.0f / s[3], as_float_i(desc->sphere_mat[p]));
                prims[3 * i + 2] = make_float4(0, 0, 0, 0);
                normals[i] = make_float4(0, 0, 0, as_float_i(~desc->sphere_mat[p]));   // ~material: a sphere
            } else {
                const int64_t j = p - ns;
                const float* t = desc->tris + 9 * j;
                prims[3 * i] = make_float4(t[0], t[1], t[2], as_float_i(p));
                prims[3 * i + 1] = make_float4(t[3], t[4], t[5], as_float_i(desc->tri_mat[j]));
                prims[3 * i + 2] = make_float4(t[6], t[7], t[8], 0.0f);
                // geometric normal in FP64, rounded once
                const double e1[3] = {(double)t[3] - t[0], (double)t[4] - t[1], (double)t[5] - t[2]};
                const double e2[3] = {(double)t[6] - t[0], (double)t[7] - t[1], (double)t[8] - t[2]};
                double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                               e1[0] * e2[1] - e1[1] * e2[0]};
                const double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
                if (l > 0)
                    for (double& x : n) x /= l;
                normals[i] = make_float4((float)n[0], (float)n[1], (float)n[2], as_float_i(desc->tri_mat[j]));
            }
        }
        float4* planes = reinterpret_cast<float4*>(base + h.off_planes);
        int* pmat = reinterpret_cast<int*>(base + h.off_plane_mat);
        for (int64_t k = 0; k < np; ++k) {
            const float* p = desc->planes + 4 * k;
            planes[k] = make_float4(p[0], p[1], p[2], p[3]);
            pmat[k] = desc->plane_mat[k];
        }
        DevMaterial* mats = reinterpret_cast<DevMaterial*>(base + h.off_mats);
        for (int m = 0; m < nm; ++m) {
            const rt_material& M = desc->materials[m];
            mats[m].a = make_float4(M.albedo[0], M.albedo[1], M.albedo[2], M.k_a);
            mats[m].b = make_float4(M.k_d, M.k_s, M.shininess, M.k_r);
            mats[m].c = make_float4(M.ior, (float)M.type, 0.0f, 0.0f);
        }
        DevLight* lights = reinterpret_cast<DevLight*>(base + h.off_lights);
        for (int l = 0; l < nl; ++l) {
            const rt_light& L = desc->lights[l];
            lights[l].pos = make_float4(L.pos[0], L.pos[1], L.pos[2], (float)L.shape);
            lights[l].intensity = make_float4(L.intensity[0], L.intensity[1], L.intensity[2], 0.0f);
            const bool area = L.shape != RT_LIGHT_POINT;
            lights[l].u = area ? make_float4(L.u[0], L.u[1], L.u[2], 0.0f) : make_float4(0, 0, 0, 0);
            lights[l].v = area ? make_float4(L.v[0], L.v[1], L.v[2], 0.0f) : make_float4(0, 0, 0, 0);
        }
        rt_scene_info& I = h.info;
        I.n_nodes = h.n_nodes;
        I.depth = h.depth;
        I.stack_size = h.stack_size;
        I.n_leaves = B.leaves;
        I.n_bvh_prims = nb;
        I.sah_cost = root.empty() ? 0.0 : B.sah_sum / std::max(root.area(), 1e-30);
        I.build_seconds = std::chrono::duration<double>(t1 - t0).count();
        for (int k = 0; k < 3; ++k) {
            I.bounds_lo[k] = root.lo[k];
            I.bounds_hi[k] = root.hi[k];
        }
        I.node_layout = o.node_layout;
        h.uid = g_scene_uid.fetch_add(1);
        h.bvh2 = std::move(nodes);
        refit_schedule(h);
        rt_scene* s = new rt_scene;
        s->h = std::move(h);
        *out = s;
        return RT_OK;
    } catch (const std::exception& e) {
        set_error(std::string("rt_build_scene: ") + e.what());
        return RT_ERR_INVALID_ARG;
    }
}

void rt_destroy_scene(rt_scene* scene) { delete scene; }

rt_status rt_scene_get_info(const rt_scene* scene, rt_scene_info* out) {
    if (!scene || !out) {
        set_error("rt_scene_get_info: NULL argument");
        return RT_ERR_INVALID_ARG;
    }
    *out = scene->h.info;
    return RT_OK;
}

rt_status rt_scene_set_layout(rt_scene* scene, int32_t node_layout) {
    if (!scene || node_layout < RT_LAYOUT_DFS || node_layout > RT_LAYOUT_BVH4Q) {
        set_error("rt_scene_set_layout: NULL scene or unknown node layout");
        return RT_ERR_INVALID_ARG;
    }
    try {
        SceneHost& h = scene->h;
        std::vector<uint8_t> node_bytes;
        int64_t n_nodes = 0;
        int stack_size = 0;
        if (!layout_nodes(h.bvh2, node_layout, h.depth, node_bytes, n_nodes, stack_size)) {
            set_error("rt_scene_set_layout: four-wide traversal stack would exceed " + std::to_string(kMaxStack) +
                      " entries");
            return RT_ERR_BVH_DEPTH;
        }
        // new blob: the node section, then every later section moved by the same amount
        const size_t tail = h.blob.size() - h.off_prims;
        const size_t new_prims = align256(node_bytes.size());
        std::vector<uint8_t> blob(new_prims + tail, 0);
        std::memcpy(blob.data(), node_bytes.data(), node_bytes.size());
        std::memcpy(blob.data() + new_prims, h.blob.data() + h.off_prims, tail);
        const size_t old_prims = h.off_prims;
        for (size_t* o : {&h.off_prims, &h.off_normals, &h.off_planes, &h.off_plane_mat, &h.off_mats, &h.off_lights,
                          &h.off_refit})
            *o = *o - old_prims + new_prims;
        h.blob.swap(blob);
        h.n_nodes = n_nodes;
        h.stack_size = stack_size;
        h.layout = node_layout;
        refit_schedule(h);
        h.info.node_layout = node_layout;
        h.info.n_nodes = n_nodes;
        h.info.stack_size = stack_size;
        h.dev = nullptr;
        h.dev_bytes = 0;
        h.uid = g_scene_uid.fetch_add(1);
        return RT_OK;
    } catch (const std::exception& e) {
        set_error(std::string("rt_scene_set_layout: ") + e.what());
        return RT_ERR_INVALID_ARG;
    }
}

size_t rt_scene_device_bytes(const rt_scene* scene) { return scene ? scene->h.blob.size() : 0; }

rt_status rt_scene_upload(rt_scene* scene, void* dev_ptr, size_t bytes, void* stream) {
    if (!scene || !dev_ptr) {
        set_error("rt_scene_upload: NULL argument");
        return RT_ERR_INVALID_ARG;
    }
    if (bytes < scene->h.blob.size()) {
        set_error("rt_scene_upload: buffer smaller than rt_scene_device_bytes");
        return RT_ERR_CAPACITY;
    }
    if (reinterpret_cast<uintptr_t>(dev_ptr) & 255) {
        set_error("rt_scene_upload: device pointer must be 256-byte aligned");
        return RT_ERR_INVALID_ARG;
    }
    hipError_t e = hipMemcpyAsync(dev_ptr, scene->h.blob.data(), scene->h.blob.size(), hipMemcpyHostToDevice,
                                  (hipStream_t)stream);
    if (e != hipSuccess) {
        set_error(std::string("rt_scene_upload: ") + hipGetErrorString(e));
        return RT_ERR_HIP;
    }
    scene->h.dev = dev_ptr;
    scene->h.dev_bytes = bytes;
    return RT_OK;
}

}  // extern "C"

namespace {
struct HostStack {
    int32_t v[kMaxStack];
    int sp = 0;
    static bool wave_all(bool v) { return v; }   // one ray at a time
    void reset() {
        v[0] = kStackDone;
        sp = 1;
    }
    void push(int32_t x) { v[sp++] = x; }
    int32_t pop() { return v[--sp]; }
};
}  // namespace

extern "C" rt_status rt_host_trace(const rt_scene* scene, const float* rays, int64_t n, int32_t any_hit, float* t,
                                   int32_t* id, uint32_t* work, int32_t nthreads) {
    if (!scene || (n > 0 && (!rays || !t || !id)) || n < 0) {
        set_error("rt_host_trace: invalid argument");
        return RT_ERR_INVALID_ARG;
    }
    const DevScene s = scene->h.host_view();
    if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
    std::atomic<int64_t> next{0};
    auto worker = [&]() {
        HostStack stk;
        for (;;) {
            const int64_t b = next.fetch_add(256);
            if (b >= n) break;
            for (int64_t i = b; i < std::min(n, b + 256); ++i) {
                const float* R = rays + 8 * i;
                const TRay r = make_tray(v3(R[0], R[1], R[2]), v3(R[3], R[4], R[5]));
                const float tmax = (R[7] > 0.0f) ? R[7] : INFINITY;
                Work w{0, 0, 0};
                Hit h = any_hit ? traverse<true, true>(s, r, tmax, stk, w) : traverse<false, true>(s, r, tmax, stk, w);
                t[i] = h.prim >= 0 ? h.t : INFINITY;
                id[i] = h.prim >= 0 ? h.id : -1;
                if (work) {
                    work[3 * i] = w.nodes;
                    work[3 * i + 1] = w.tris;
                    work[3 * i + 2] = w.spheres;
                }
            }
        }
    };
    std::vector<std::thread> th;
    for (int k = 1; k < nthreads; ++k) th.emplace_back(worker);
    worker();
    for (auto& x : th) x.join();
    return RT_OK;
}
