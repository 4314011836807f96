// bvh_quant.h -- 8-bit quantization of a four-wide node's child boxes
// (RT_LAYOUT_BVH4Q), shared by the host build and the device refit so that
// both produce the same bits from the same boxes.
#pragma once

#include "rt_common.h"

namespace mirt {

// Per axis: scale 2^e, the smallest power of two with 255 * 2^e >= the
// node's extent; the node stores the scale s = 4 * 2^e (as its exponent e + 2
// in a signed byte) and the origin p = the lowest child plane m minus
// 1024 * 2^e (rounded, then lowered an ulp at a time until q = 0 decodes to
// at most m), so that byte q decodes to the plane fma(256 + q / 4, s, p) =
// p + (1024 + q) 2^e: the value 256 + q / 4 is exact in FP16, which the
// device traversal widens two bytes at a time.  A lower plane takes the largest q whose decoded value is <= the
// true plane, an upper plane the smallest q whose decoded value is >= it
// (checked with that same fma), so every decoded box contains its child's
// padded box.  lo/hi: child boxes; valid: used slots; child: the four
// references.  Returns false if an axis cannot be covered (non-finite
// extents).
HD bool quantize_children(const float (&lo)[4][3], const float (&hi)[4][3], const bool (&valid)[4], int4 child,
                          Node4q& q) {
#pragma clang fp contract(off)
    float p[3] = {0.0f, 0.0f, 0.0f};
    uint32_t ebytes = 0, qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        float mn = INFINITY, mx = -INFINITY;
        for (int i = 0; i < 4; ++i)
            if (valid[i]) {
                mn = lo[i][a] < mn ? lo[i][a] : mn;
                mx = hi[i][a] > mx ? hi[i][a] : mx;
            }
        if (!(mn <= mx)) {
            mn = 0.0f;
            mx = 0.0f;
        }
        const double ext = (double)mx - mn;
        int e = -126;
        if (ext > 0.0) {
            // ceil(log2(ext / 255)) exactly: v = m 2^x with m in [0.5, 1)
            int x = 0;
            const double m = frexp(ext / 255.0, &x);
            const int c = m == 0.5 ? x - 1 : x;
            e = c > -126 ? c : -126;
        }
        for (;; ++e) {
            if (e > 125) return false;
            const float sc = as_float_i((e + 127) << 23);       // 2^e, a normal float
            const float s4 = as_float_i((e + 129) << 23);       // the stored scale 4 * 2^e
            float org = (float)((double)mn - 1024.0 * (double)sc);
            while (fmaf(256.0f, s4, org) > mn) org = nextafterf(org, -INFINITY);
            p[a] = org;
            bool ok = true;
            uint32_t wl = 0, wh = 0;
            for (int i = 0; i < 4 && ok; ++i) {
                if (!valid[i]) {   // an unused slot decodes to an inverted box (low plane above high)
                    wl |= 255u << (8 * i);
                    continue;
                }
                double ql = floor(((double)lo[i][a] - mn) / sc);
                ql = ql > 0.0 ? (ql < 255.0 ? ql : 255.0) : 0.0;
                while (ql > 0.0 && fmaf(256.0f + 0.25f * (float)ql, s4, org) > lo[i][a]) ql -= 1.0;
                double qh = ceil(((double)hi[i][a] - mn) / sc);
                qh = qh > 0.0 ? qh : 0.0;
                while (qh <= 255.0 && fmaf(256.0f + 0.25f * (float)qh, s4, org) < hi[i][a]) qh += 1.0;
                if (qh > 255.0 || ql > 255.0) ok = false;
                wl |= (uint32_t)ql << (8 * i);
                wh |= (uint32_t)qh << (8 * i);
            }
            if (ok) {
                ebytes |= (uint32_t)(uint8_t)(int8_t)(e + 2) << (8 * a);
                qlo[a] = wl;
                qhi[a] = wh;
                break;
            }
        }
    }
    uint32_t mask = 0;
    for (int i = 0; i < 4; ++i) mask |= valid[i] ? (1u << i) : 0u;
    ebytes |= mask << 24;
    q.origin = make_float4(p[0], p[1], p[2], as_float_i((int)ebytes));
    q.qa = make_uint4(qlo[0], qhi[0], qlo[1], qhi[1]);
    q.qb = make_uint4(qlo[2], qhi[2], (uint32_t)child.x, (uint32_t)child.y);
    q.qc = make_int4(child.z, child.w, 0, 0);
    return true;
}

}  // namespace mirt
