// refit.cpp -- BVH refit on the GPU: new positions for an uploaded scene's
// spheres and triangles, the same tree.  Rewrites the device blob's primitive
// records and triangle normals, then every node's child boxes level by level,
// deepest level first (the refit order stored in the blob), so that dynamic
// scenes need no host rebuild between frames.
//
// Boxes follow the host build exactly: a leaf's box is the union of its
// primitives' boxes (triangle: vertex min/max; sphere: centre -+ r), padded
// outward by 2^-19 of the scene scale (max(1, max |coordinate|, max |c| + r));
// an inner child's box is the union of its children's padded boxes, which is
// the padded union in FP32 as well (x - pad is monotone in x).  Quantized
// nodes are requantized with the build's quantizer.  Refitting a scene to its
// own positions therefore reproduces the uploaded blob bit for bit.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "bvh_quant.h"
#include "mirt_internal.h"

namespace mirt {
namespace {

// workspace words
constexpr int kRefitStatus = 0;   // non-zero: invalid input, nothing was changed
constexpr int kRefitScale = 1;    // float bits of the new scene scale (all values >= 1: uint order = float order)
constexpr size_t kRefitHeader = 256;

__global__ void k_refit_init(uint32_t* ws) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ws[kRefitStatus] = 0u;
        ws[kRefitScale] = __float_as_uint(1.0f);
    }
}

// Validity and scale of the new positions (caller order).
__global__ void k_refit_scan(const float* sph, int64_t ns, const float* tri, int64_t nt, uint32_t* ws) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float m = 1.0f;
    bool bad = false;
    if (i < ns) {
        const float* s = sph + 4 * i;
        for (int k = 0; k < 4; ++k) bad = bad || !isfinite(s[k]);
        bad = bad || !(s[3] > 0.0f);
        if (!bad)
            for (int k = 0; k < 3; ++k) m = fmaxf(m, fabsf(s[k]) + s[3]);
    } else if (i < ns + nt) {
        const float* t = tri + 9 * (i - ns);
        for (int k = 0; k < 9; ++k) {
            bad = bad || !isfinite(t[k]);
            if (!bad) m = fmaxf(m, fabsf(t[k]));
        }
    }
    if (bad) atomicOr(ws + kRefitStatus, 1u);
    else if (m > 1.0f) atomicMax(ws + kRefitScale, __float_as_uint(m));
}

// Primitive records in leaf order from the new positions (ids and materials kept).
__global__ void k_refit_prims(float4* prims, float4* normals, int64_t nb, int32_t ns, const float* sph,
                              const float* tri, const uint32_t* ws) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb || ws[kRefitStatus]) return;
    const float4 p0 = prims[3 * i], p1 = prims[3 * i + 1];
    const int32_t p = as_int_f(p0.w);
    if (p < ns) {
        const float* s = sph + 4 * p;
        const float r = s[3];
        prims[3 * i] = make_float4(s[0], s[1], s[2], p0.w);
        prims[3 * i + 1] = make_float4(r, r * r, __frcp_rn(r), p1.w);
        return;
    }
    const float* t = tri + 9 * (int64_t)(p - ns);
    prims[3 * i] = make_float4(t[0], t[1], t[2], p0.w);
    prims[3 * i + 1] = make_float4(t[3], t[4], t[5], p1.w);
    prims[3 * i + 2] = make_float4(t[6], t[7], t[8], 0.0f);
    // geometric normal in FP64, rounded once (as the build)
    const double e1[3] = {(double)t[3] - t[0], (double)t[4] - t[1], (double)t[5] - t[2]};
    const double e2[3] = {(double)t[6] - t[0], (double)t[7] - t[1], (double)t[8] - t[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (l > 0)
        for (double& x : n) x /= l;
    normals[i] = make_float4((float)n[0], (float)n[1], (float)n[2], p1.w);   // w: the material, as built
}

struct RBox {
    float lo[3], hi[3];
};

__device__ __forceinline__ void rb_empty(RBox& b) {
    for (int k = 0; k < 3; ++k) {
        b.lo[k] = INFINITY;
        b.hi[k] = -INFINITY;
    }
}
__device__ __forceinline__ void rb_grow(RBox& b, const RBox& c) {
    for (int k = 0; k < 3; ++k) {
        b.lo[k] = c.lo[k] < b.lo[k] ? c.lo[k] : b.lo[k];
        b.hi[k] = c.hi[k] > b.hi[k] ? c.hi[k] : b.hi[k];
    }
}

// Box of child reference ref: a leaf's padded primitive union, an inner
// node's box from the side array; empty for an empty leaf.
__device__ RBox child_box(int32_t ref, const float4* prims, int32_t ns, const float* side, float pad) {
    RBox b;
    rb_empty(b);
    if (ref >= 0) {
        for (int k = 0; k < 3; ++k) {
            b.lo[k] = side[6 * (int64_t)ref + k];
            b.hi[k] = side[6 * (int64_t)ref + 3 + k];
        }
        return b;
    }
    const int32_t first = leaf_first(ref), cnt = leaf_count(ref);
    if (cnt == 0) return b;
    for (int32_t i = first; i < first + cnt; ++i) {
        const float4 p0 = prims[3 * i], p1 = prims[3 * i + 1];
        RBox c;
        if (as_int_f(p0.w) < ns) {
            const float v[3] = {p0.x, p0.y, p0.z};
            for (int k = 0; k < 3; ++k) {
                c.lo[k] = v[k] - p1.x;
                c.hi[k] = v[k] + p1.x;
            }
        } else {
            const float4 p2 = prims[3 * i + 2];
            const float x[3] = {p0.x, p1.x, p2.x}, y[3] = {p0.y, p1.y, p2.y}, z[3] = {p0.z, p1.z, p2.z};
            const float* a[3] = {x, y, z};
            for (int k = 0; k < 3; ++k) {
                c.lo[k] = a[k][0];
                c.hi[k] = a[k][0];
                for (int v = 1; v < 3; ++v) {
                    c.lo[k] = a[k][v] < c.lo[k] ? a[k][v] : c.lo[k];
                    c.hi[k] = a[k][v] > c.hi[k] ? a[k][v] : c.hi[k];
                }
            }
        }
        rb_grow(b, c);
    }
    for (int k = 0; k < 3; ++k) {
        b.lo[k] -= pad;
        b.hi[k] += pad;
    }
    return b;
}

// One level of the refit order.  KIND: 0 binary nodes, 1 four-wide float, 2 quantized four-wide.
template <int KIND>
__global__ void k_refit_level(uint8_t* nodes, const float4* prims, int32_t ns, const int32_t* order, int64_t count,
                              float* side, uint32_t* ws) {
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count || ws[kRefitStatus]) return;
    const float pad = __uint_as_float(ws[kRefitScale]) * 0x1p-19f;
    const int32_t me = order[t];
    RBox all;
    rb_empty(all);
    if (KIND == 0) {
        Node& n = reinterpret_cast<Node*>(nodes)[me];
        const RBox l = child_box(n.d.x, prims, ns, side, pad), r = child_box(n.d.y, prims, ns, side, pad);
        n.a = make_float4(l.lo[0], l.hi[0], l.lo[1], l.hi[1]);
        n.b = make_float4(r.lo[0], r.hi[0], r.lo[1], r.hi[1]);
        n.c = make_float4(l.lo[2], l.hi[2], r.lo[2], r.hi[2]);
        rb_grow(all, l);
        rb_grow(all, r);
    } else {
        int4 child;
        if (KIND == 1) {
            child = reinterpret_cast<const Node4*>(nodes)[me].child;
        } else {
            const Node4q& q = reinterpret_cast<const Node4q*>(nodes)[me];
            child = make_int4((int32_t)q.qb.z, (int32_t)q.qb.w, q.qc.x, q.qc.y);
        }
        const int32_t c[4] = {child.x, child.y, child.z, child.w};
        float lo[4][3], hi[4][3];
        bool valid[4];
        for (int s = 0; s < 4; ++s) {
            // an empty leaf is an unused slot (all-+inf box, not in the valid mask)
            valid[s] = !(c[s] < 0 && leaf_count(c[s]) == 0);
            const RBox b = child_box(c[s], prims, ns, side, pad);
            for (int k = 0; k < 3; ++k) {
                lo[s][k] = valid[s] ? b.lo[k] : INFINITY;
                hi[s][k] = valid[s] ? b.hi[k] : INFINITY;
            }
            if (valid[s]) rb_grow(all, b);
        }
        if (KIND == 1) {
            Node4& n = reinterpret_cast<Node4*>(nodes)[me];
            n.lox = make_float4(lo[0][0], lo[1][0], lo[2][0], lo[3][0]);
            n.hix = make_float4(hi[0][0], hi[1][0], hi[2][0], hi[3][0]);
            n.loy = make_float4(lo[0][1], lo[1][1], lo[2][1], lo[3][1]);
            n.hiy = make_float4(hi[0][1], hi[1][1], hi[2][1], hi[3][1]);
            n.loz = make_float4(lo[0][2], lo[1][2], lo[2][2], lo[3][2]);
            n.hiz = make_float4(hi[0][2], hi[1][2], hi[2][2], hi[3][2]);
        } else {
            Node4q q;
            if (!quantize_children(lo, hi, valid, child, q)) {
                // non-finite extents (cannot follow a valid input): no child is entered
                q.origin = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                q.qa = make_uint4(0, 0, 0, 0);
                q.qb = make_uint4(0, 0, (uint32_t)child.x, (uint32_t)child.y);
                q.qc = make_int4(child.z, child.w, 0, 0);
                atomicOr(ws + kRefitStatus, 2u);
            }
            reinterpret_cast<Node4q*>(nodes)[me] = q;
        }
    }
    for (int k = 0; k < 3; ++k) {
        side[6 * (int64_t)me + k] = all.lo[k];
        side[6 * (int64_t)me + 3 + k] = all.hi[k];
    }
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t refit_scratch_bytes(const SceneHost& h) {
    return kRefitHeader + a256(24 * (size_t)std::max<int64_t>(h.n_nodes, 1));
}

// Scratch of rt_scene_refit_noalloc: the refit header and a box per node in
// one file-scope device array.  Every GPU the library runs on holds its own
// copy until the process ends; calls on one GPU share it.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
__device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current.  In host code `scratch` names a host-side stand-in,
// never a device address: only this pointer is passed to kernels.
rt_status scratch_ptr(const char* who, uint8_t** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* per_dev[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error(std::string(who) + ": hipGetDevice: " + hipGetErrorString(e));
        return RT_ERR_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error(std::string(who) + ": device index beyond 63");
        return RT_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> g(mu);
    if (!per_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string(who) + ": hipGetSymbolAddress(scratch): " + hipGetErrorString(e));
            return RT_ERR_HIP;
        }
        per_dev[dev] = p;
    }
    *out = static_cast<uint8_t*>(per_dev[dev]);
    return RT_OK;
}

// Argument checks shared by both entry points (everything but the scratch).
rt_status refit_check(const char* who, const rt_scene* scene, const float* spheres, const float* tris) {
    if (!scene) {
        set_error(std::string(who) + ": NULL scene");
        return RT_ERR_INVALID_ARG;
    }
    const SceneHost& h = scene->h;
    if (!h.dev) {
        set_error(std::string(who) + ": scene not uploaded (call rt_scene_upload)");
        return RT_ERR_NOT_UPLOADED;
    }
    if ((h.n_spheres && !spheres) || (h.n_tris && !tris)) {
        set_error(std::string(who) + ": NULL position array with a non-zero count");
        return RT_ERR_INVALID_ARG;
    }
    if (h.refit_levels.size() < 2 || h.refit_levels.back() != h.n_nodes) {
        set_error(std::string(who) + ": scene has no refit order");
        return RT_ERR_INVALID_ARG;
    }
    return RT_OK;
}

// The refit itself on a checked scene and a scratch of refit_scratch_bytes (256-byte aligned).
rt_status refit_enqueue(rt_scene* scene, const float* spheres, const float* tris, void* workspace, int32_t flags,
                        void* stream) {
    SceneHost& h = scene->h;
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t* base = static_cast<uint8_t*>(h.dev);
    uint32_t* ws = static_cast<uint32_t*>(workspace);
    float* side = reinterpret_cast<float*>(static_cast<uint8_t*>(workspace) + kRefitHeader);
    const int64_t ns = h.n_spheres, nt = h.n_tris, nb = ns + nt;
    hipLaunchKernelGGL(k_refit_init, dim3(1), dim3(64), 0, st, ws);
    if (nb > 0) {
        const unsigned g = (unsigned)((nb + 255) / 256);
        hipLaunchKernelGGL(k_refit_scan, dim3(g), dim3(256), 0, st, spheres, ns, tris, nt, ws);
        hipLaunchKernelGGL(k_refit_prims, dim3(g), dim3(256), 0, st, reinterpret_cast<float4*>(base + h.off_prims),
                           reinterpret_cast<float4*>(base + h.off_normals), nb, (int32_t)ns, spheres, tris, ws);
    }
    const int32_t* order = reinterpret_cast<const int32_t*>(base + h.off_refit);
    const float4* prims = reinterpret_cast<const float4*>(base + h.off_prims);
    uint8_t* nodes = base + h.off_nodes;
    for (size_t l = 0; l + 1 < h.refit_levels.size(); ++l) {
        const int64_t lo = h.refit_levels[l], n = h.refit_levels[l + 1] - lo;
        if (n <= 0) continue;
        const dim3 g((unsigned)((n + 255) / 256)), b(256);
        if (h.layout == RT_LAYOUT_BVH4Q)
            hipLaunchKernelGGL(k_refit_level<2>, g, b, 0, st, nodes, prims, (int32_t)ns, order + lo, n, side, ws);
        else if (h.layout == RT_LAYOUT_BVH4)
            hipLaunchKernelGGL(k_refit_level<1>, g, b, 0, st, nodes, prims, (int32_t)ns, order + lo, n, side, ws);
        else
            hipLaunchKernelGGL(k_refit_level<0>, g, b, 0, st, nodes, prims, (int32_t)ns, order + lo, n, side, ws);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("rt_scene_refit: ") + hipGetErrorString(e));
        return RT_ERR_HIP;
    }
    if (flags & RT_FLAG_SYNC) {
        uint32_t status = 0;
        e = hipMemcpyAsync(&status, ws + kRefitStatus, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            set_error(std::string("rt_scene_refit: ") + hipGetErrorString(e));
            return RT_ERR_HIP;
        }
        if (status) {
            set_error("rt_scene_refit: non-finite position or radius <= 0; the scene was left unchanged");
            return RT_ERR_INVALID_ARG;
        }
    }
    return RT_OK;
}

}  // namespace
}  // namespace mirt

using namespace mirt;

extern "C" {

size_t rt_scene_refit_workspace_bytes(const rt_scene* scene) {
    if (!scene) return 0;
    return refit_scratch_bytes(scene->h);
}

rt_status rt_scene_refit(rt_scene* scene, const float* spheres, const float* tris, void* workspace,
                         size_t workspace_bytes, int32_t flags, void* stream) {
    rt_status rs = refit_check("rt_scene_refit", scene, spheres, tris);
    if (rs != RT_OK) return rs;
    if (!workspace || workspace_bytes < refit_scratch_bytes(scene->h)) {
        set_error("rt_scene_refit: workspace missing or smaller than rt_scene_refit_workspace_bytes");
        return RT_ERR_CAPACITY;
    }
    if (reinterpret_cast<uintptr_t>(workspace) & 255) {
        set_error("rt_scene_refit: workspace must be 256-byte aligned");
        return RT_ERR_INVALID_ARG;
    }
    return refit_enqueue(scene, spheres, tris, workspace, flags, stream);
}

size_t rt_scene_refit_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

rt_status rt_scene_refit_noalloc(rt_scene* scene, const float* spheres, const float* tris, int32_t flags,
                                 void* stream) {
    if (scene && refit_scratch_bytes(scene->h) > kNoAllocScratchBytes) {
        set_error("rt_scene_refit_noalloc: the scene's " + std::to_string(scene->h.n_nodes) +
                  " nodes need " + std::to_string(refit_scratch_bytes(scene->h)) +
                  " bytes of scratch, more than the " + std::to_string(kNoAllocScratchBytes) +
                  " bytes the library holds per GPU (use rt_scene_refit with a workspace)");
        return RT_ERR_CAPACITY;
    }
    rt_status rs = refit_check("rt_scene_refit_noalloc", scene, spheres, tris);
    if (rs != RT_OK) return rs;
    uint8_t* ptr = nullptr;
    rs = scratch_ptr("rt_scene_refit_noalloc", &ptr);
    if (rs != RT_OK) return rs;
    return refit_enqueue(scene, spheres, tris, ptr, flags, stream);
}

}  // extern "C"
