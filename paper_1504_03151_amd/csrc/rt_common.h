// rt_common.h -- data layouts and the FP32 intersection / traversal code shared
// by the gfx950 kernels and the library's host-side FP32 traversal.
//
// Method (arXiv 1504.03151): closest hit of a ray over all objects and the
// any-hit shadow query of Algorithm 1 (Section III); the sphere is the
// quadratic of Eq. 9-12 (Section IV.B).  The acceleration structure (a binary
// BVH), triangles and planes extend the paper's sphere-only scenes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef HD
#define HD __host__ __device__ __forceinline__
#endif

namespace mirt {

// ---------------------------------------------------------------------------
// layouts
// ---------------------------------------------------------------------------
// BVH node: 64 bytes holding the boxes of BOTH children, so one node fetch
// (four 16-byte loads) tests two boxes.
//   a = (L.lo.x, L.hi.x, L.lo.y, L.hi.y)
//   b = (R.lo.x, R.hi.x, R.lo.y, R.hi.y)
//   c = (L.lo.z, L.hi.z, R.lo.z, R.hi.z)
//   d = (left, right, 0, 0)
// A child reference >= 0 is an inner node index; < 0 is a leaf ~((first << 4) | count),
// count in [1, 15] primitives in leaf order.  A reference with count 0 is empty.
struct alignas(16) Node {
    float4 a, b, c;
    int4 d;
};
static_assert(sizeof(Node) == 64, "node must be 64 bytes");

// Four-wide node (RT_LAYOUT_BVH4): 128 bytes, one L2 line, holding the boxes of
// up to four children in SoA form (component i of each float4 is child i).
// An unused slot has an all-+inf box, which no slab test accepts, and an empty
// leaf reference.  Built on the host by collapsing the binary tree.
struct alignas(128) Node4 {
    float4 lox, hix, loy, hiy, loz, hiz;
    int4 child;
    int4 pad;
};
static_assert(sizeof(Node4) == 128, "four-wide node must be 128 bytes");

// Quantized four-wide node (RT_LAYOUT_BVH4Q): 64 bytes.  Child box planes are
// 8-bit codes q on a grid of step 2^e per axis: plane = fma(256 + q / 4, s, p)
// with the stored scale s = 4 * 2^e and origin p (the lowest child plane less
// 1024 * 2^e, so that the code's value 256 + q / 4 is exact in FP16); the
// builder chooses each q so that the decoded box contains the child's
// (padded) box, so traversal stays exact and only visits a little more.
//   origin = (p.x, p.y, p.z, bits: exponents of s_x | s_y << 8 | s_z << 16 (signed bytes) | valid-child mask << 24)
//   qa = (lo.x, hi.x, lo.y, hi.y) with byte i = child i
//   qb = (lo.z, hi.z, child 0, child 1)
//   qc = (child 2, child 3, 0, 0)
struct alignas(64) Node4q {
    float4 origin;
    uint4 qa;
    uint4 qb;
    int4 qc;
};
static_assert(sizeof(Node4q) == 64, "quantized four-wide node must be 64 bytes");

constexpr int kLeafBits = 4;
constexpr int kLeafMaxCount = 15;
constexpr int32_t kStackDone = INT32_MIN;
constexpr int kMaxStack = 96;

HD int32_t leaf_ref(int32_t first, int32_t count) { return ~((first << kLeafBits) | count); }
HD int32_t leaf_first(int32_t ref) { return (~ref) >> kLeafBits; }
HD int32_t leaf_count(int32_t ref) { return (~ref) & ((1 << kLeafBits) - 1); }

// Primitive record in leaf order, 48 bytes (three float4):
//   triangle: (v0, id) (v1, mat) (v2, 0)
//   sphere:   (c, id)  (r, r^2, 0, mat) (0)
// id = original id as int bits (spheres 0..ns-1, then triangles); a record is
// a sphere iff id < n_spheres.
struct alignas(16) DevMaterial {
    float4 a;  // albedo.rgb, k_a
    float4 b;  // k_d, k_s, shininess, k_r
    float4 c;  // ior, type, 0, 0
};

struct alignas(16) DevLight {
    float4 pos;        // xyz; w = shape (RT_LIGHT_*) as a float
    float4 intensity;
    float4 u, v;       // area lights: edge or semi-axis vectors
};

// Device view of one scene (pointers into the uploaded blob).
struct DevScene {
    const Node* nodes;
    const Node4* nodes4;      // the same section, when wide == 1
    const Node4q* nodes4q;    // the same section, when wide == 2
    int wide;                 // 0 binary nodes; 1 four-wide (RT_LAYOUT_BVH4); 2 quantized four-wide (RT_LAYOUT_BVH4Q)
    const float4* prims;      // [n_bvh * 3]
    const float4* normals;    // [n_bvh]  triangle: unit geometric normal (FP64 on host, rounded), material (bits);
                              //          sphere: 0, 0, 0, ~material (bits)
    const float4* planes;     // [n_planes] (n, h): n.x = h
    const int* plane_mat;     // [n_planes]
    const DevMaterial* mats;
    const DevLight* lights;
    int n_spheres, n_tris, n_planes, n_lights;
    int n_bvh;                // n_spheres + n_tris
    int stack_size;           // traversal stack entries needed (tree depth + 2)
};

// Hit codes: -1 miss; [0, n_bvh) BVH primitive in leaf order; n_bvh + k plane k.

// ---------------------------------------------------------------------------
// small vector helpers
// ---------------------------------------------------------------------------
struct V3 {
    float x, y, z;
};
HD V3 v3(float x, float y, float z) { return V3{x, y, z}; }
HD V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
HD V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
HD V3 operator*(V3 a, float s) { return v3(a.x * s, a.y * s, a.z * s); }
HD V3 operator*(float s, V3 a) { return v3(a.x * s, a.y * s, a.z * s); }
HD V3 operator-(V3 a) { return v3(-a.x, -a.y, -a.z); }
HD float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
HD V3 mul(V3 a, V3 b) { return v3(a.x * b.x, a.y * b.y, a.z * b.z); }
HD float maxabs(V3 a) { return fmaxf(fabsf(a.x), fmaxf(fabsf(a.y), fabsf(a.z))); }
HD float sel(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
HD V3 xyz(float4 f) { return v3(f.x, f.y, f.z); }

HD float min3f(float a, float b, float c) { return fminf(a, fminf(b, c)); }
HD float max3f(float a, float b, float c) { return fmaxf(a, fmaxf(b, c)); }

HD float as_float_i(int i) {
    union { int i; float f; } u;
    u.i = i;
    return u.f;
}
HD int as_int_f(float f) {
    union { float f; int i; } u;
    u.f = f;
    return u.i;
}

// ---------------------------------------------------------------------------
// ray prepared for traversal
// ---------------------------------------------------------------------------
struct TRay {
    V3 o, d;
    V3 inv;     // 1/d with zero components replaced by a tiny signed value
    V3 oinv;    // o * inv
    int kx, ky, kz;
    float sx, sy, sz;  // shear of the watertight triangle test
};

HD TRay make_tray(V3 o, V3 d) {
    TRay r;
    r.o = o;
    r.d = d;
    const float tiny = 1e-20f;
    float ix = fabsf(d.x) > tiny ? d.x : copysignf(tiny, d.x);
    float iy = fabsf(d.y) > tiny ? d.y : copysignf(tiny, d.y);
    float iz = fabsf(d.z) > tiny ? d.z : copysignf(tiny, d.z);
    r.inv = v3(1.0f / ix, 1.0f / iy, 1.0f / iz);
    r.oinv = mul(o, r.inv);
    // watertight test (Woop, Benthin, Wald, JCGT 2013): dominant axis kz,
    // winding-preserving permutation, shear that maps the ray to +z.
    const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    const float dz = sel(d, kz);
    if (dz < 0.0f) {
        int t = kx;
        kx = ky;
        ky = t;
    }
    r.kx = kx;
    r.ky = ky;
    r.kz = kz;
    r.sx = sel(d, kx) / dz;
    r.sy = sel(d, ky) / dz;
    r.sz = 1.0f / dz;
    return r;
}

// Slab test of both children of a node.  Boxes are padded outward by the
// builder, so the FP32 test never rejects a box the ray truly crosses.
// Slab test of one child of a four-wide node, same arithmetic as box2.
HD bool box1(const TRay& r, float lx, float hx, float ly, float hy, float lz, float hz, float tbest, float& tn) {
    const float x0 = fmaf(lx, r.inv.x, -r.oinv.x), x1 = fmaf(hx, r.inv.x, -r.oinv.x);
    const float y0 = fmaf(ly, r.inv.y, -r.oinv.y), y1 = fmaf(hy, r.inv.y, -r.oinv.y);
    const float z0 = fmaf(lz, r.inv.z, -r.oinv.z), z1 = fmaf(hz, r.inv.z, -r.oinv.z);
    const float tmin = max3f(fminf(x0, x1), fminf(y0, y1), fmaxf(fminf(z0, z1), 0.0f));
    const float tmax = min3f(fmaxf(x0, x1), fmaxf(y0, y1), fminf(fmaxf(z0, z1), tbest));
    tn = tmin;
    return tmin <= tmax;
}

HD void box2(const TRay& r, float4 a, float4 b, float4 c, float tbest, bool& hitL, bool& hitR, float& tl,
             float& tr) {
    const float lx0 = fmaf(a.x, r.inv.x, -r.oinv.x), lx1 = fmaf(a.y, r.inv.x, -r.oinv.x);
    const float ly0 = fmaf(a.z, r.inv.y, -r.oinv.y), ly1 = fmaf(a.w, r.inv.y, -r.oinv.y);
    const float lz0 = fmaf(c.x, r.inv.z, -r.oinv.z), lz1 = fmaf(c.y, r.inv.z, -r.oinv.z);
    const float rx0 = fmaf(b.x, r.inv.x, -r.oinv.x), rx1 = fmaf(b.y, r.inv.x, -r.oinv.x);
    const float ry0 = fmaf(b.z, r.inv.y, -r.oinv.y), ry1 = fmaf(b.w, r.inv.y, -r.oinv.y);
    const float rz0 = fmaf(c.z, r.inv.z, -r.oinv.z), rz1 = fmaf(c.w, r.inv.z, -r.oinv.z);
    const float lmin = max3f(fminf(lx0, lx1), fminf(ly0, ly1), fmaxf(fminf(lz0, lz1), 0.0f));
    const float lmax = min3f(fmaxf(lx0, lx1), fmaxf(ly0, ly1), fminf(fmaxf(lz0, lz1), tbest));
    const float rmin = max3f(fminf(rx0, rx1), fminf(ry0, ry1), fmaxf(fminf(rz0, rz1), 0.0f));
    const float rmax = min3f(fmaxf(rx0, rx1), fmaxf(ry0, ry1), fminf(fmaxf(rz0, rz1), tbest));
    hitL = lmin <= lmax;
    hitR = rmin <= rmax;
    tl = lmin;
    tr = rmin;
}

// Watertight ray/triangle test (Woop, Benthin, Wald 2013).  Edge functions are
// evaluated without contraction so a shared edge gives exactly opposite values
// in its two triangles; an exact zero is re-evaluated in double, as that paper
// prescribes.  Two-sided; returns t in (0, +inf) or -1.
HD float tri_t(const TRay& r, float4 p0, float4 p1, float4 p2) {
#pragma clang fp contract(off)
    const V3 A = xyz(p0) - r.o, B = xyz(p1) - r.o, C = xyz(p2) - r.o;
    const float Az = sel(A, r.kz), Bz = sel(B, r.kz), Cz = sel(C, r.kz);
    const float Ax = sel(A, r.kx) - r.sx * Az, Ay = sel(A, r.ky) - r.sy * Az;
    const float Bx = sel(B, r.kx) - r.sx * Bz, By = sel(B, r.ky) - r.sy * Bz;
    const float Cx = sel(C, r.kx) - r.sx * Cz, Cy = sel(C, r.ky) - r.sy * Cz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return -1.0f;
    const float det = U + V + W;
    if (det == 0.0f) return -1.0f;
    const float T = U * (r.sz * Az) + V * (r.sz * Bz) + W * (r.sz * Cz);
    if ((det > 0.0f && T <= 0.0f) || (det < 0.0f && T >= 0.0f)) return -1.0f;
    return T / det;
}

// Ray/sphere (Eq. 11-12), evaluated in the cancellation-free form of Haines,
// Guenther and Akenine-Moller ("Precision Improvements for Ray/Sphere
// Intersection", Ray Tracing Gems, 2019): the discriminant r^2 - |f - (f.d)d|^2
// and the root pair q, c'/q.  d must be unit length.  Returns the smallest
// root in (0, +inf) or -1.
HD float sphere_t(const TRay& r, float4 p0, float4 p1) {
    const V3 f = r.o - xyz(p0);
    const float bq = -dot(f, r.d);                 // t of closest approach
    const V3 l = f + bq * r.d;                     // centre -> closest point
    const float disc = p1.y - dot(l, l);           // r^2 - |l|^2
    if (disc < 0.0f) return -1.0f;
    const float cc = dot(f, f) - p1.y;             // c' = |o-c|^2 - r^2
    const float q = bq + copysignf(sqrtf(disc), bq);
    if (q == 0.0f) return -1.0f;
    float t0 = cc / q, t1 = q;
    if (t0 > t1) {
        const float t = t0;
        t0 = t1;
        t1 = t;
    }
    if (t0 > 0.0f) return t0;
    if (t1 > 0.0f) return t1;
    return -1.0f;
}

HD float plane_t(const TRay& r, float4 pl) {
    const V3 n = xyz(pl);
    const float nd = dot(n, r.d);
    if (nd == 0.0f) return -1.0f;
    const float t = (pl.w - dot(n, r.o)) / nd;
    return t > 0.0f ? t : -1.0f;
}

// ---------------------------------------------------------------------------
// traversal
// ---------------------------------------------------------------------------
struct Hit {
    float t;
    int prim;   // hit code (see above)
    int id;     // original id, for the tie-break and the id output
};

struct Work {
    uint32_t nodes, tris, spheres;
};

// Tests the primitives of one leaf; true when an any-hit query is answered.
template <bool ANY, bool COUNT>
HD bool leaf_hits(const DevScene& s, const TRay& r, int32_t leaf, Hit& h, Work& work) {
    const int32_t first = leaf_first(leaf), cnt = leaf_count(leaf);
    for (int i = first; i < first + cnt; ++i) {
        const float4 p0 = s.prims[3 * i];
        const int id = as_int_f(p0.w);
        float t;
        if (id < s.n_spheres) {
            if (COUNT) work.spheres++;
            t = sphere_t(r, p0, s.prims[3 * i + 1]);
        } else {
            if (COUNT) work.tris++;
            t = tri_t(r, p0, s.prims[3 * i + 1], s.prims[3 * i + 2]);
        }
        if (t > 0.0f && (t < h.t || (t == h.t && h.prim >= 0 && id < h.id))) {
            h.t = t;
            h.prim = i;
            h.id = id;
            if (ANY) return true;
        }
    }
    return false;
}

template <bool ANY, bool COUNT, class Stack>
HD bool trace_bvh2(const DevScene& s, const TRay& r, Hit& h, Stack& stk, Work& work) {
    // While-while traversal with postponed leaves: a lane that reaches a leaf
    // keeps it and goes on descending until every active lane of the wave
    // holds a leaf (Stack::wave_all), then the wave tests leaves together, so
    // fewer lanes idle in the primitive loop.  Leaf order changes the work,
    // never the result (closest hit with the id tie-break, or any hit).
    stk.reset();
    int32_t node = 0, leaf = 0;   // leaf 0 = none (the root is always an inner node)
    while (node != kStackDone) {
        while (node >= 0) {
            const Node* n = s.nodes + node;
            const float4 a = n->a, b = n->b, c = n->c;
            const int4 d = n->d;
            if (COUNT) work.nodes++;
            bool hl, hr;
            float tl, tr;
            box2(r, a, b, c, h.t, hl, hr, tl, tr);
            int32_t cl = d.x, cr = d.y;
            if (hl && hr) {
                if (tr < tl) {
                    const int32_t t = cl;
                    cl = cr;
                    cr = t;
                }
                stk.push(cr);
                node = cl;
            } else if (hl) {
                node = cl;
            } else if (hr) {
                node = cr;
            } else {
                node = stk.pop();
            }
            if (node < 0 && node != kStackDone && leaf == 0) {
                leaf = node;
                node = stk.pop();
            }
            if (Stack::wave_all(leaf != 0)) break;
        }
        while (leaf != 0) {
            if (leaf_hits<ANY, COUNT>(s, r, leaf, h, work)) return true;
            if (node < 0 && node != kStackDone) {
                leaf = node;
                node = stk.pop();
            } else {
                leaf = 0;
            }
        }
    }
    return false;
}

HD void cswap(float& ka, int32_t& ca, float& kb, int32_t& cb) {
    if (kb < ka) {
        const float k = ka;
        ka = kb;
        kb = k;
        const int32_t c = ca;
        ca = cb;
        cb = c;
    }
}

// Four-wide traversal: the hit children of a node are ordered by entry
// distance (five-comparator network, misses sorted last), the far ones pushed,
// the nearest taken next; leaves are postponed as in the binary traversal.
// Distance along the ray to the plane of byte q of a quantized plane word.
// The node stores per axis a scale s = 4 * 2^e and an origin p such that the
// plane is p + (256 + q / 4) s; the distance (p + (256 + q / 4) s - o) / d is
// one fma, (256 + q / 4) a + b, with a = s / d and b = (p - o) / d per node
// and axis.  The folded form differs from decoding the plane first by a few
// FP32 roundings of quantities bounded by the coordinate magnitude (p lies
// about four node extents below the node), far inside the builder's outward
// padding of 2^-19 of the scene scale, so the test stays conservative.
// 256 + q / 4 is exact in FP16 (the spacing in [256, 512) is 1/4): the device
// widens two bytes at a time into FP16 halves with one byte permute and takes
// the widening into a mixed-precision fma; the host evaluates the same fma on
// the same operands in FP32.
HD float qdist(uint32_t w, int i, float a, float b) {
    return fmaf(256.0f + 0.25f * (float)((w >> (8 * i)) & 0xFFu), a, b);
}
#if defined(__HIP_DEVICE_COMPILE__)
typedef _Float16 mirt_half2 __attribute__((ext_vector_type(2)));
// bytes 0 and 1 (k = 0) or 2 and 3 (k = 1) of w as the FP16 halves 256 + q / 4 (0x5C00 | q is
// 256 + q / 4: exponent 8, q in the top eight of the ten mantissa bits)
__device__ __forceinline__ uint32_t qhalves(uint32_t w, int k) {
    return __builtin_amdgcn_perm(0x5C5C5C5Cu, w, k ? 0x04030402u : 0x04010400u);
}
__device__ __forceinline__ float qdist_h(uint32_t pr, int h, float a, float b) {
    return fmaf((float)__builtin_bit_cast(mirt_half2, pr)[h], a, b);
}
#endif

// Children of a quantized four-wide node: folded plane distances, then the
// slab test.  Per axis the plane word nearer along the ray (the low planes
// when the direction component is non-negative, else the high ones) is picked
// once per node, so each child's entry is a max and its exit a min of three
// distances with no per-axis min/max (the same result: for a valid child the
// low plane is not above the high one, and no distance is NaN).
HD void kids_q(const Node4q* n, const TRay& r, float tbest, bool& b0, bool& b1, bool& b2, bool& b3, float& k0,
               float& k1, float& k2, float& k3, int4& ch) {
    const float4 o = n->origin;
    const uint4 qa = n->qa, qb = n->qb;
    const int4 qc = n->qc;
    const uint32_t eb = (uint32_t)as_int_f(o.w);
    // a = s / d = 2^n / d with the signed exponent bytes n (exact, like the product by 2^n)
    const float ax = ldexpf(r.inv.x, (int)(int8_t)(eb & 0xFFu)), ay = ldexpf(r.inv.y, (int)(int8_t)((eb >> 8) & 0xFFu)),
                az = ldexpf(r.inv.z, (int)(int8_t)((eb >> 16) & 0xFFu));
    const float bx = fmaf(o.x, r.inv.x, -r.oinv.x), by = fmaf(o.y, r.inv.y, -r.oinv.y),
                bz = fmaf(o.z, r.inv.z, -r.oinv.z);
    const bool px = r.inv.x >= 0.0f, py = r.inv.y >= 0.0f, pz = r.inv.z >= 0.0f;
    const uint32_t nx = px ? qa.x : qa.y, fx = px ? qa.y : qa.x;
    const uint32_t ny = py ? qa.z : qa.w, fy = py ? qa.w : qa.z;
    const uint32_t nz = pz ? qb.x : qb.y, fz = pz ? qb.y : qb.x;
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t nx2[2] = {qhalves(nx, 0), qhalves(nx, 1)}, fx2[2] = {qhalves(fx, 0), qhalves(fx, 1)};
    const uint32_t ny2[2] = {qhalves(ny, 0), qhalves(ny, 1)}, fy2[2] = {qhalves(fy, 0), qhalves(fy, 1)};
    const uint32_t nz2[2] = {qhalves(nz, 0), qhalves(nz, 1)}, fz2[2] = {qhalves(fz, 0), qhalves(fz, 1)};
#define MIRT_QD(w, i, a, b) qdist_h(w##2[(i) >> 1], (i) & 1, a, b)
#else
#define MIRT_QD(w, i, a, b) qdist(w, i, a, b)
#endif
#define MIRT_QCHILD(i, b, k)                                                                              \
    {                                                                                                     \
        const float tn = max3f(MIRT_QD(nx, i, ax, bx), MIRT_QD(ny, i, ay, by), fmaxf(MIRT_QD(nz, i, az, bz), 0.0f)); \
        const float tf = min3f(MIRT_QD(fx, i, ax, bx), MIRT_QD(fy, i, ay, by), fminf(MIRT_QD(fz, i, az, bz), tbest)); \
        k = tn;                                                                                           \
        b = tn <= tf;                                                                                     \
    }
    MIRT_QCHILD(0, b0, k0)
    MIRT_QCHILD(1, b1, k1)
    MIRT_QCHILD(2, b2, k2)
    MIRT_QCHILD(3, b3, k3)
#undef MIRT_QCHILD
#undef MIRT_QD
    ch = make_int4((int)qb.z, (int)qb.w, qc.x, qc.y);
}

HD void kids_f(const Node4* n, const TRay& r, float tbest, bool& b0, bool& b1, bool& b2, bool& b3, float& k0,
               float& k1, float& k2, float& k3, int4& ch) {
    const float4 lx = n->lox, hx = n->hix, ly = n->loy, hy = n->hiy, lz = n->loz, hz = n->hiz;
    ch = n->child;
    b0 = box1(r, lx.x, hx.x, ly.x, hy.x, lz.x, hz.x, tbest, k0);
    b1 = box1(r, lx.y, hx.y, ly.y, hy.y, lz.y, hz.y, tbest, k1);
    b2 = box1(r, lx.z, hx.z, ly.z, hy.z, lz.z, hz.z, tbest, k2);
    b3 = box1(r, lx.w, hx.w, ly.w, hy.w, lz.w, hz.w, tbest, k3);
}

template <bool ANY, bool COUNT, bool QUANT, class Stack>
HD bool trace_bvh4(const DevScene& s, const TRay& r, Hit& h, Stack& stk, Work& work) {
    stk.reset();
    int32_t node = 0, leaf = 0;
    while (node != kStackDone) {
        while (node >= 0) {
            if (COUNT) work.nodes++;
            bool b0, b1, b2, b3;
            float k0, k1, k2, k3;
            int4 ch;
            if (QUANT) kids_q(s.nodes4q + node, r, h.t, b0, b1, b2, b3, k0, k1, k2, k3, ch);
            else kids_f(s.nodes4 + node, r, h.t, b0, b1, b2, b3, k0, k1, k2, k3, ch);
            if (!(b0 || b1 || b2 || b3)) {
                node = stk.pop();
            } else {
                // missed children sort last with key +inf; the entry distance of a box the ray
                // reaches is finite (+inf means parallel to a slab and outside it), so after the
                // sort "key < +inf" marks the children to visit
                int32_t c0 = ch.x, c1 = ch.y, c2 = ch.z, c3 = ch.w;
                k0 = b0 ? k0 : INFINITY;
                k1 = b1 ? k1 : INFINITY;
                k2 = b2 ? k2 : INFINITY;
                k3 = b3 ? k3 : INFINITY;
                cswap(k0, c0, k1, c1);
                cswap(k2, c2, k3, c3);
                cswap(k0, c0, k2, c2);
                cswap(k1, c1, k3, c3);
                cswap(k1, c1, k2, c2);
                if (k3 < INFINITY) stk.push(c3);
                if (k2 < INFINITY) stk.push(c2);
                if (k1 < INFINITY) stk.push(c1);
                node = c0;
            }
            if (node < 0 && node != kStackDone && leaf == 0) {
                leaf = node;
                node = stk.pop();
            }
            if (Stack::wave_all(leaf != 0)) break;
        }
        while (leaf != 0) {
            if (leaf_hits<ANY, COUNT>(s, r, leaf, h, work)) return true;
            if (node < 0 && node != kStackDone) {
                leaf = node;
                node = stk.pop();
            } else {
                leaf = 0;
            }
        }
    }
    return false;
}

// Closest hit (ANY = false) or any hit (ANY = true) in (0, tmax).  Ties in t
// go to the smaller original id.  Stack is a small push/pop policy object
// (LDS-resident on the GPU, an array on the host).
// L selects the node layout at compile time (0 binary, 1 four-wide float, 2
// four-wide quantized), or at run time from s.wide when L < 0.
template <bool ANY, bool COUNT, int L = -1, class Stack>
HD Hit traverse(const DevScene& s, const TRay& r, float tmax, Stack& stk, Work& work) {
    Hit h;
    h.t = tmax;
    h.prim = -1;
    h.id = -1;
    for (int k = 0; k < s.n_planes; ++k) {
        const float t = plane_t(r, s.planes[k]);
        const int id = s.n_bvh + k;
        if (t > 0.0f && (t < h.t || (t == h.t && h.prim >= 0 && id < h.id))) {
            h.t = t;
            h.prim = s.n_bvh + k;
            h.id = id;
            if (ANY) return h;
        }
    }
    const int wide = L >= 0 ? L : s.wide;
    if (wide == 2) trace_bvh4<ANY, COUNT, true>(s, r, h, stk, work);
    else if (wide == 1) trace_bvh4<ANY, COUNT, false>(s, r, h, stk, work);
    else trace_bvh2<ANY, COUNT>(s, r, h, stk, work);
    return h;
}

// ---------------------------------------------------------------------------
// counter-based jitter: the 32-bit PCG hash of Jarzynski and Olano, "Hash
// Functions for GPU Rendering", JCGT 9(3), 2020.
// ---------------------------------------------------------------------------
HD uint32_t pcg_hash(uint32_t v) {
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

HD double jitter01(uint64_t seed, uint32_t frame, uint32_t pixel, uint32_t s, uint32_t dim) {
    uint32_t h = pcg_hash((uint32_t)seed);
    h = pcg_hash(h ^ (uint32_t)(seed >> 32));
    h = pcg_hash(h ^ frame);
    h = pcg_hash(h ^ pixel);
    h = pcg_hash(h ^ (s * 2u + dim));
    return (double)(h >> 8) * (1.0 / 16777216.0);
}

// Random number k of the path bounce at `depth` of sample s of a pixel (global
// illumination): the jitter chain through the pixel, then the sample, then a
// word with the top bit set (no jitter word has it) holding depth and k.
// 24 bits, exact as a float.
HD float path_rand(uint64_t seed, uint32_t frame, uint32_t pixel, uint32_t s, uint32_t depth, uint32_t k) {
    uint32_t h = pcg_hash((uint32_t)seed);
    h = pcg_hash(h ^ (uint32_t)(seed >> 32));
    h = pcg_hash(h ^ frame);
    h = pcg_hash(h ^ pixel);
    h = pcg_hash(h ^ s);
    h = pcg_hash(h ^ (0x80000000u | (depth << 2) | k));
    return (float)(h >> 8) * (1.0f / 16777216.0f);
}

}  // namespace mirt
