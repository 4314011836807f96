// render.cpp -- gfx950 wavefront kernels and the rt_render / rt_intersect /
// rt_occluded launchers.
//
// One frame (Section IV.A: the recursion runs as iterations; Section V: each
// pass adds its colour into the pixels):
//   acc = 0
//   for each pass of samples:
//     raygen               -> ray queue Q0 (SoA)
//     for depth k = 0..D:
//       extend  (Q_k)      -> hit buffer      closest hit, BVH in HBM, stack in LDS
//       shade   (Q_k, H)   -> acc += w*local-ambient/bg; shadow queue S; Q_{k+1}
//       shadow  (S)        -> acc += contribution of unblocked lights
//   resolve                -> out_rgb = acc / spp
// Queue tails live in device counters, so no step reads anything back to the
// host and the whole frame can be captured in a HIP graph and replayed.
#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "mirt_internal.h"

namespace mirt {

#define HIP_TRY(x)                                                                   \
    do {                                                                             \
        hipError_t err_ = (x);                                                       \
        if (err_ != hipSuccess) {                                                    \
            set_error(std::string(#x) + ": " + hipGetErrorString(err_));            \
            return RT_ERR_HIP;                                                       \
        }                                                                            \
    } while (0)

// ---------------------------------------------------------------------------
// queues
// ---------------------------------------------------------------------------
// A queued ray is three 16-byte records: a traversal lane reads its ray with
// two loads.  meta: depth (bits 0-3) | sample (bits 4-19) | scene (bits 20-31).
struct RayQ {
    float4* a;   // origin, pixel (bits; kDeadRay for an empty slot)
    float4* b;   // unit direction, meta (bits)
    float4* c;   // path weight rgb, unused
};
// A shadow entry is three 16-byte records, so that a traversal lane reads its
// segment with two loads and, if unblocked, its contribution with one.
struct ShadowQ {
    float4* a;       // origin (the light point), tmax
    float4* b;       // unit direction, scene of the entry (bits; batched frames)
    float4* c;       // contribution rgb, pixel (bits)
    uint32_t* key;   // bin of each entry (deferred shadows: light and origin cell), or NULL
};
struct HitQ {
    float* t;
    int* prim;
};

// counters (uint32) inside the workspace, reset at the start of each pass
constexpr int kCtrRays = 0;       // [16] rays queued at depth k
constexpr int kCtrRayCur = 16;    // [16] extend fetch cursors
constexpr int kCtrShadow = 32;    // [16] shadow rays queued at depth k
constexpr int kCtrShadowCur = 48; // [16] shadow fetch cursors
constexpr int kCtrStatus = 64;    // overflow flags
constexpr int kCtrDead = 65;      // padding slots of ragged tiles in the primary queue
constexpr int kCtrShadowAll = 66; // shadow rays of every depth of a pass (deferred shadow traversal)
constexpr int kCtrShadowAllCur = 67;
constexpr int kCtrWords = 128;     // words cleared at the start of every pass
constexpr int kCtrFrame = 128;     // frame number, written by the host before each launch
constexpr int kCtrAccum = 130;     // frames already in the accumulator (progressive mode), written likewise
constexpr int kCtrRec = 129;       // learned form: cache queries recorded this frame (cleared per frame)
// XCD-aware fetching: each fetch cursor above (kCtrRayCur .. kCtrShadowAllCur) is backed by kXcd segment
// cursors, kXcdStride words apart, in the block at kCtrXcd (cleared with the counters).
constexpr int kXcd = 8;            // XCDs of the chip; workgroups are dispatched to them round-robin
constexpr int kXcdStride = 16;
constexpr int kCtrXcd = 256;
constexpr int kCurSlots = kCtrShadowAllCur - kCtrRayCur + 1;
constexpr int kCtrTotal = kCtrXcd + kCurSlots * kXcd * kXcdStride;

// the segment cursors of fetch cursor c (one of kCtrRayCur + k, kCtrShadowCur + k, kCtrShadowAllCur)
__host__ __device__ inline uint32_t* xcd_cursor(uint32_t* ctr, int c) {
    return ctr + kCtrXcd + (c - kCtrRayCur) * kXcd * kXcdStride;
}

struct CamConst {
    double eye[3], f[3], r[3], u[3];
    double th, aspect;
    int W, H, spp, jitter, m;   // m = sqrt(spp) when spp is a perfect square > 1, else 0
    int tw_log2;                // a wave's pixel tile is 2^tw_log2 wide and 64 / 2^tw_log2 high
    uint32_t frame;
    uint64_t seed;
};

// pixel tile of one wave's primary rays: log2 of its width (height = 64 / width)
static int tile_log2w(int tile) {
    static const int lw[4] = {3, 4, 5, 2};   // RT_TILE_8X8, 16X4, 32X2, 4X16
    return lw[tile & 3];
}
static bool tile_ok(int tile) { return tile >= RT_TILE_8X8 && tile <= RT_TILE_4X16; }
static int64_t tiles_x_of(int width, int tile) {
    const int w = 1 << tile_log2w(tile);
    return (width + w - 1) / w;
}
static int64_t tiles_y_of(int height, int tile) {
    const int h = 64 >> tile_log2w(tile);
    return (height + h - 1) / h;
}

struct ShadeConst {
    float bg[3];
    float eps;
    int max_depth;
    int spp;
    uint32_t qcap, scap;
    int per_sample;     // accumulation slot = pixel * spp + sample instead of pixel
    uint32_t acc_off;   // first accumulation slot of the scene
    int32_t* out_ids;   // [H][W][spp] or NULL
    int defer_shadow;   // 1: shadow rays of all depths go to one queue, traced after the last bounce
    uint64_t seed;      // hash seed of the frame (area-light sample points)
    const float4* light_pts;   // [spp][n_lights] sample points of the frame's passes, or NULL (point lights)
    // deferred shadows are binned by (light, origin cell) before they are traced:
    // cell = floor((x - bin_lo) * bin_inv) per axis on a bin_c^3 grid over the scene
    float bin_lo[3], bin_inv[3];
    int bin_c;
    int gi;   // 1: global illumination, one randomly chosen continuation per hit (path tracing)
    int sum_depth0;   // 1: the four waves of a block at depth 0 are four samples of one pixel tile
};

// One scene of a batched frame (device table, one entry per scene).
struct BatchScene {
    DevScene sc;
    ShadeConst shc;
    CamConst cam;
    uint32_t ray_off, n_rays;   // primary-ray slots [ray_off, ray_off + n_rays)
    uint32_t n_acc;             // accumulation slots [shc.acc_off, shc.acc_off + n_acc)
    int tiles_x;
    float inv_spp;
    float* out_rgb;
    uint32_t lpt_first, lpt_count;   // area lights: entries of the batch's light-point table
};

template <bool BATCH>
__device__ __forceinline__ const DevScene& scene_of(const DevScene& single, const BatchScene* tab, uint32_t sid) {
    return BATCH ? tab[sid].sc : single;
}
template <bool BATCH>
__device__ __forceinline__ const ShadeConst& shade_of(const ShadeConst& single, const BatchScene* tab, uint32_t sid) {
    return BATCH ? tab[sid].shc : single;
}

// ---------------------------------------------------------------------------
// wave helpers (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// exclusive prefix sum of v over the wave; total in *tot (all lanes must call)
__device__ __forceinline__ uint32_t wave_scan(uint32_t v, uint32_t& tot) {
    uint32_t x = v;
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    tot = __shfl(x, 63, 64);
    return x - v;
}

// reserve n_lane slots per lane in a queue with one atomic per wave; returns
// the lane's first slot (all lanes must call)
__device__ __forceinline__ uint32_t wave_reserve(uint32_t n_lane, uint32_t* tail) {
    uint32_t tot;
    const uint32_t off = wave_scan(n_lane, tot);
    uint32_t base = 0;
    if (lane_id() == 0 && tot) base = atomicAdd(tail, tot);
    base = __shfl(base, 0, 64);
    return base + off;
}

struct LdsStack {
    int32_t* p;   // this lane's column
    int sp;
    static __device__ bool wave_all(bool v) { return __all(v); }
    __device__ void reset() {
        p[0] = kStackDone;
        sp = 1;
    }
    __device__ void push(int32_t v) {
        p[sp * 64] = v;
        ++sp;
    }
    __device__ int32_t pop() {
        --sp;
        return p[sp * 64];
    }
};

__device__ __forceinline__ LdsStack lds_stack(int32_t* smem, int stack_size) {
    LdsStack s;
    s.p = smem + (threadIdx.x >> 6) * stack_size * 64 + (threadIdx.x & 63);
    s.sp = 0;
    return s;
}

// Traversal stack of the frame kernels: the top kSplitLds entries of each lane
// live in LDS ([entry][lane] columns), deeper entries (rare: only on long
// paths of deep trees) in a per-thread global region ([entry][thread]).
// Keeping LDS at 4 KB per wave lets register pressure, not LDS, set occupancy.
constexpr int kSplitLds = 16;
// The LDS column is typed with the LDS address space: given two generic
// pointers, the compiler merges the two loads of a pop into one flat load
// through a selected pointer, which waits on the vector memory counter and
// occupies the texture address unit even when every lane reads LDS.
typedef __attribute__((address_space(3))) int32_t lds_i32;
struct SplitStack {
    lds_i32* p;      // LDS column of this lane
    int32_t* g;      // overflow column of this thread (stride = threads of the grid)
    uint32_t gstride;
    int sp;
    static __device__ bool wave_all(bool v) { return __all(v); }   // every active lane of the wave
    __device__ void reset() {
        p[0] = kStackDone;
        sp = 1;
    }
    __device__ void push(int32_t v) {
        if (sp < kSplitLds) p[sp * 64] = v;
        else g[(size_t)(sp - kSplitLds) * gstride] = v;
        ++sp;
    }
    __device__ int32_t pop() {
        --sp;
        int32_t v = p[min(sp, kSplitLds - 1) * 64];
        if (sp >= kSplitLds) v = g[(size_t)(sp - kSplitLds) * gstride];
        return v;
    }
};

__device__ __forceinline__ SplitStack split_stack(int32_t* smem, int32_t* overflow) {
    SplitStack s;
    s.p = (lds_i32*)(smem + (threadIdx.x >> 6) * kSplitLds * 64 + (threadIdx.x & 63));
    s.gstride = gridDim.x * blockDim.x;
    s.g = overflow + blockIdx.x * blockDim.x + threadIdx.x;
    s.sp = 0;
    return s;
}

template <bool COUNT>
__device__ __forceinline__ void flush_work(const Work& w, unsigned long long* dst) {
    if (!COUNT || !dst) return;
    uint32_t tn, tt, tsph;
    wave_scan(w.nodes, tn);
    wave_scan(w.tris, tt);
    wave_scan(w.spheres, tsph);
    if (lane_id() == 0) {
        atomicAdd(dst + 0, (unsigned long long)tn);
        atomicAdd(dst + 1, (unsigned long long)tt);
        atomicAdd(dst + 2, (unsigned long long)tsph);
    }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_zero_u32(uint32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Clear a pass's counters and the XCD segment cursors of its fetch cursors.
static void clear_counters(uint32_t* ctr, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kCtrWords), 0, st, ctr, kCtrWords);
    constexpr int n = kCtrTotal - kCtrXcd;
    hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256), dim3(256), 0, st, ctr + kCtrXcd, n);
}

// Ray slots of a pass map 1:1 to threads: a wave covers one 64-pixel tile
// (8x8, 16x4, 32x2 or 4x16) of one sample, so primary rays of a wave are
// coherent and no atomic is needed.
// Lanes past the image edge (ragged tiles) write a dead ray (pixel kDeadRay)
// that the later stages skip.  The camera ray is formed in FP64 and rounded
// once to FP32.
constexpr uint32_t kDeadRay = 0xFFFFFFFFu;

// Primary ray for slot `slot` = local thread index `g` of a pass over one
// scene (64-pixel tiles, samples s0 .. s0 + ns - 1).  Returns false for a dead
// padding slot.
// The root node's child boxes against a ray, in the traversal's own arithmetic (closest hit, no bound on t):
// false when no child box is reached, so that the traversal, starting there, would find nothing (BVH
// primitives only; the caller rules out planes).
template <int L>
__device__ __forceinline__ bool root_reached(const DevScene& s, const TRay& r) {
    if (L == 0) {
        const Node* n = s.nodes;
        bool hl, hr;
        float tl, tr;
        box2(r, n->a, n->b, n->c, INFINITY, hl, hr, tl, tr);
        return hl || hr;
    }
    bool b0, b1, b2, b3;
    float k0, k1, k2, k3;
    int4 ch;
    if (L == 2) kids_q(s.nodes4q, r, INFINITY, b0, b1, b2, b3, k0, k1, k2, k3, ch);
    else kids_f(s.nodes4, r, INFINITY, b0, b1, b2, b3, k0, k1, k2, k3, ch);
    return b0 || b1 || b2 || b3;
}

// What ray generation did with a slot.
enum GenKind { kGenDead = 0, kGenQueued = 1, kGenMissed = 2 };

// L >= 0 (scenes without planes): a camera ray that misses every child box of
// the root can hit nothing; it is not queued (its slot is marked like a dead
// one, which the later stages skip) and the caller adds its background term.
template <int L = -1>
__device__ __forceinline__ GenKind gen_ray(const CamConst& cam, uint32_t frame, int s0, int ns, int tiles_x, uint32_t g,
                                           int per_sample, uint32_t acc_off, uint32_t meta_hi, RayQ q, uint32_t slot,
                                           const DevScene* sc = nullptr, uint32_t* pix_out = nullptr,
                                           uint32_t* sample_out = nullptr) {
    const uint32_t lane = g & 63u;
    const uint32_t tile_sample = g >> 6;
    const uint32_t tile = tile_sample / (uint32_t)ns;
    const int s = s0 + (int)(tile_sample - tile * (uint32_t)ns);
    const uint32_t ty = tile / (uint32_t)tiles_x;
    const int lw = cam.tw_log2;
    const int px = ((int)(tile - ty * (uint32_t)tiles_x) << lw) + (int)(lane & ((1u << lw) - 1u));
    const int py = ((int)ty << (6 - lw)) + (int)(lane >> lw);
    if (px >= cam.W || py >= cam.H) {
        q.a[slot].w = as_float_i((int)kDeadRay);
        return kGenDead;
    }
    const uint32_t pixel = (uint32_t)py * cam.W + px;
    double jx = 0.5, jy = 0.5, xi0 = 0.5, xi1 = 0.5;
    if (cam.jitter) {
        xi0 = jitter01(cam.seed, frame, pixel, (uint32_t)s, 0);
        xi1 = jitter01(cam.seed, frame, pixel, (uint32_t)s, 1);
    }
    if (cam.m > 0) {
        jx = ((double)(s % cam.m) + xi0) / cam.m;
        jy = ((double)(s / cam.m) + xi1) / cam.m;
    } else {
        jx = xi0;
        jy = xi1;
    }
    const double X = (2.0 * ((double)px + jx) / cam.W - 1.0) * cam.aspect * cam.th;
    const double Y = (1.0 - 2.0 * ((double)py + jy) / cam.H) * cam.th;
    double d[3];
    for (int i = 0; i < 3; ++i) d[i] = cam.f[i] + X * cam.r[i] + Y * cam.u[i];
    const double inv = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const uint32_t pix = acc_off + (per_sample ? pixel * (uint32_t)cam.spp + (uint32_t)s : pixel);
    const V3 o = v3((float)cam.eye[0], (float)cam.eye[1], (float)cam.eye[2]);
    const V3 dir = v3((float)(d[0] * inv), (float)(d[1] * inv), (float)(d[2] * inv));
    if (L >= 0 && !root_reached<L>(*sc, make_tray(o, dir))) {
        q.a[slot].w = as_float_i((int)kDeadRay);
        *pix_out = pix;
        *sample_out = pixel * (uint32_t)cam.spp + (uint32_t)s;
        return kGenMissed;
    }
    q.a[slot] = make_float4(o.x, o.y, o.z, as_float_i((int)pix));
    q.b[slot] = make_float4(dir.x, dir.y, dir.z, as_float_i((int)(meta_hi | ((uint32_t)s << 4))));
    q.c[slot] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
    return kGenQueued;
}

__device__ __forceinline__ void count_dead(bool dead, uint32_t* ctr) {
    const uint64_t m = __ballot(dead);
    if (m && (threadIdx.x & 63u) == (uint32_t)(__ffsll((unsigned long long)m) - 1))
        atomicAdd(ctr + kCtrDead, (uint32_t)__popcll(m));
}

// Adds each thread's term to its pixel of acc.  In ray generation order lane l
// of a block's four waves is one pixel in four samples: then the four terms
// are summed and added once, each of three waves adding one channel; a group
// whose pixels differ adds its terms one by one.  All threads of the block
// must call; lds_add and lds_pix are the block's shared arrays.
__device__ __forceinline__ void add_block_terms(float* acc, bool has, uint32_t pix, V3 add, float (&lds_add)[3][256],
                                                uint32_t (&lds_pix)[256]) {
    lds_pix[threadIdx.x] = has ? pix : kDeadRay;
    lds_add[0][threadIdx.x] = add.x;
    lds_add[1][threadIdx.x] = add.y;
    lds_add[2][threadIdx.x] = add.z;
    __syncthreads();
    if (threadIdx.x < 192) {   // wave c adds channel c
        const uint32_t c = threadIdx.x >> 6, l = threadIdx.x & 63u, q0 = lds_pix[l];
        const bool same =
            q0 != kDeadRay && lds_pix[64 + l] == q0 && lds_pix[128 + l] == q0 && lds_pix[192 + l] == q0;
        if (same) {
            atomicAdd(acc + 3 * q0 + c, (lds_add[c][l] + lds_add[c][64 + l]) + (lds_add[c][128 + l] + lds_add[c][192 + l]));
        } else {
            for (int k = 0; k < 4; ++k) {
                const uint32_t q = lds_pix[64 * k + l];
                if (q == kDeadRay) continue;
                atomicAdd(acc + 3 * q + c, lds_add[c][64 * k + l]);
            }
        }
    }
}

// Camera rays that ray generation finishes itself (RootMiss, when L >= 0): the
// background term goes to acc (weight 1) and -1 to the hit ids.
struct RootMiss {
    float* acc;
    int32_t* out_ids;   // [pixels][spp] or NULL
    float bg[3];
};

// L < 0: every live slot is queued.  L >= 0 (the node layout; scenes without
// planes): rays that miss the root's child boxes are finished here and count
// as traced rays, not as dead slots.
template <int L>
__global__ __launch_bounds__(256) void k_raygen(CamConst cam, int s0, int ns, int tiles_x, uint32_t n_threads,
                                                RayQ q, uint32_t* ctr, uint32_t cap, int per_sample, DevScene sc,
                                                RootMiss rm) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) {
        ctr[kCtrRays] = min(n_threads, cap);
        if (n_threads > cap) atomicOr(ctr + kCtrStatus, 1u);
    }
    const bool in = g < n_threads && g < cap;
    if (L < 0) {
        if (in) count_dead(gen_ray(cam, ctr[kCtrFrame], s0, ns, tiles_x, g, per_sample, 0u, 0u, q, g) == kGenDead, ctr);
        return;
    }
    __shared__ float lds_add[3][256];
    __shared__ uint32_t lds_pix[256];
    uint32_t pix = 0, sample = 0;
    const GenKind k =
        in ? gen_ray<L>(cam, ctr[kCtrFrame], s0, ns, tiles_x, g, per_sample, 0u, 0u, q, g, &sc, &pix, &sample)
           : kGenQueued;
    count_dead(k == kGenDead, ctr);
    const bool missed = k == kGenMissed;
    if (missed && rm.out_ids) rm.out_ids[sample] = -1;
    if (!__syncthreads_or(missed ? 1 : 0)) return;   // block-uniform
    add_block_terms(rm.acc, missed, pix, v3(rm.bg[0], rm.bg[1], rm.bg[2]), lds_add, lds_pix);
}

// Batched frames: one global slot space over all scenes; each thread finds
// its scene by binary search over the scenes' first slots.
__global__ __launch_bounds__(256) void k_raygen_batch(const BatchScene* tab, int n_scenes, uint32_t n_threads,
                                                      RayQ q, uint32_t* ctr, uint32_t cap) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) {
        ctr[kCtrRays] = min(n_threads, cap);
        if (n_threads > cap) atomicOr(ctr + kCtrStatus, 1u);
    }
    if (g >= n_threads || g >= cap) return;
    int lo = 0, hi = n_scenes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].ray_off <= g) lo = mid;
        else hi = mid - 1;
    }
    const BatchScene& B = tab[lo];
    const bool live = gen_ray(B.cam, B.cam.frame, 0, B.shc.spp, B.tiles_x, g - B.ray_off, B.shc.per_sample,
                              B.shc.acc_off, (uint32_t)lo << 20, q, g) != kGenDead;
    count_dead(!live, ctr);
}

// Persistent traversal kernels: each wave takes `chunk` consecutive queue
// entries per atomic on the fetch cursor (a multiple of 64) and traces them 64
// at a time until the queue is drained.
// XCD-aware queue fetch.  The queue [0, count) is cut into kXcd contiguous
// segments; a wave takes `chunk` entries at a time from the segment of its own
// XCD (blockIdx modulo kXcd), so each XCD's L2 serves rays that are adjacent in
// the queue (neighbouring pixels, or one shadow bin), then helps the other
// segments in turn until all are drained.  Wave-uniform.
struct QueueFetch {
    uint32_t* cur;   // kXcd segment cursors, kXcdStride words apart
    uint32_t count, chunk;
    int x, left;
    __device__ QueueFetch(uint32_t* c, uint32_t n, uint32_t ch)
        : cur(c), count(n), chunk(ch), x((int)(blockIdx.x % kXcd)), left(kXcd) {}
    __device__ bool next(uint32_t& base, uint32_t& end) {
        while (left > 0) {
            const uint32_t lo = (uint32_t)((uint64_t)count * x / kXcd);
            const uint32_t hi = (uint32_t)((uint64_t)count * (x + 1) / kXcd);
            uint32_t b = 0;
            if (lane_id() == 0) b = lo < hi ? atomicAdd(cur + kXcdStride * x, chunk) : hi - lo;
            b = __shfl(b, 0, 64);
            if (b < hi - lo) {
                base = lo + b;
                end = min(base + chunk, hi);
                return true;
            }
            x = x + 1 == kXcd ? 0 : x + 1;
            --left;
        }
        return false;
    }
};

template <bool COUNT, bool BATCH, int L = -1>
__device__ __forceinline__ void extend_queue(const DevScene& sc, const BatchScene* tab, const RayQ& q, const HitQ& hit,
                                             const uint32_t* count_p, uint32_t* cursor, uint32_t cap, uint32_t chunk,
                                             int32_t* overflow, unsigned long long* work_out) {
    __shared__ int32_t smem[4 * kSplitLds * 64];
    SplitStack stk = split_stack(smem, overflow);
    const uint32_t count = min(*count_p, cap);   // a producer that overflowed still bumped the tail
    Work w{0, 0, 0};
    QueueFetch f(cursor, count, chunk);
    uint32_t base, end;
    while (f.next(base, end)) {
        for (uint32_t b = base; b < end; b += 64) {
            const uint32_t i = b + lane_id();
            if (i < end) {
                const float4 ra = q.a[i];
                if ((uint32_t)as_int_f(ra.w) == kDeadRay) {
                    hit.prim[i] = -1;
                    continue;
                }
                const float4 rb = q.b[i];
                const DevScene& S = scene_of<BATCH>(sc, tab, BATCH ? ((uint32_t)as_int_f(rb.w) >> 20) : 0u);
                const TRay r = make_tray(v3(ra.x, ra.y, ra.z), v3(rb.x, rb.y, rb.z));
                const Hit h = traverse<false, COUNT, L>(S, r, INFINITY, stk, w);
                hit.t[i] = h.t;
                hit.prim[i] = h.prim;
            }
        }
    }
    flush_work<COUNT>(w, work_out);
}

// Seven waves per SIMD (at most 72 registers; the single-scene form needs 68,
// no spills; eight waves measured slower for the batched form, which shares
// this kernel).  L: the node layout compiled in (-1: read from the
// scene, as batched frames, whose scenes may differ, and counting frames do);
// a kernel built for one layout spends no registers on the others' code.
template <bool COUNT, bool BATCH, int L = -1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 7))) void k_extend(DevScene sc, const BatchScene* tab, RayQ q, HitQ hit,
                                                const uint32_t* count_p, uint32_t* cursor, uint32_t cap,
                                                uint32_t chunk, int32_t* overflow, unsigned long long* work_out) {
    extend_queue<COUNT, BATCH, L>(sc, tab, q, hit, count_p, cursor, cap, chunk, overflow, work_out);
}

// The same for the bounces after the first: their queues are small and incoherent, so a launch is bound by
// the latency of each ray's chain of node fetches; eight waves per SIMD (at most 64 registers) hide more of
// it than fewer waves with more registers.
template <int L>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_extend_deep(
    DevScene sc, RayQ q, HitQ hit, const uint32_t* count_p, uint32_t* cursor, uint32_t cap, uint32_t chunk,
    int32_t* overflow) {
    extend_queue<false, false, L>(sc, nullptr, q, hit, count_p, cursor, cap, chunk, overflow, nullptr);
}

// A record read for the last time (a shadow-queue record by the shadow
// launch; a ray and its hit by shading): non-temporal loads keep the stream
// from evicting the BVH node and queue lines that are read again from the L2.
// (The closest-hit launches read their queue normally: shading reads the same
// records right after.)
__device__ __forceinline__ float4 load_stream(const float4* p) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

// Any-hit over the shadow queue; adds the contribution of each unblocked light
// to its pixel.  Eight waves per SIMD (at most 64 registers): more rays in
// flight hide more of the node-fetch latency than fewer waves with more
// registers.
template <bool COUNT, bool BATCH, int L = -1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_shadow(DevScene sc, const BatchScene* tab, ShadowQ s,
                                                const uint32_t* count_p, uint32_t* cursor, uint32_t cap,
                                                uint32_t chunk, float* acc, int32_t* overflow,
                                                unsigned long long* work_out, const uint32_t* perm = nullptr,
                                                const uint32_t* begin_p = nullptr, uint32_t* vis = nullptr) {
    __shared__ int32_t smem[4 * kSplitLds * 64];
    SplitStack stk = split_stack(smem, overflow);
    // entries [begin, end) of the queue; with perm, perm[0, end - begin) lists them in binned order
    const uint32_t end_all = min(*count_p, cap);
    const uint32_t begin = begin_p ? min(*begin_p, end_all) : 0u;
    const uint32_t count = end_all - begin;
    Work w{0, 0, 0};
    QueueFetch f(cursor, count, chunk);
    uint32_t base, end;
    while (f.next(base, end)) {
        for (uint32_t b = base; b < end; b += 64) {
            const uint32_t j = b + lane_id();
            if (j < end) {
                const uint32_t i = perm ? __builtin_nontemporal_load(perm + j) : begin + j;   // binned order
                const float4 ea = BATCH ? s.a[i] : load_stream(s.a + i), eb = BATCH ? s.b[i] : load_stream(s.b + i);
                const DevScene& S = scene_of<BATCH>(sc, tab, BATCH ? (uint32_t)as_int_f(eb.w) : 0u);
                const TRay r = make_tray(v3(ea.x, ea.y, ea.z), v3(eb.x, eb.y, eb.z));
                const Hit h = traverse<true, COUNT, L>(S, r, ea.w, stk, w);
                if (h.prim < 0) {
                    if (vis) {   // binned order visits pixels at random: mark the entry, add in queue order later
                        atomicOr(vis + (i >> 5), 1u << (i & 31u));
                    } else {
                        const float4 ec = BATCH ? s.c[i] : load_stream(s.c + i);
                        const uint32_t p = (uint32_t)as_int_f(ec.w);
                        atomicAdd(acc + 3 * p + 0, ec.x);
                        atomicAdd(acc + 3 * p + 1, ec.y);
                        atomicAdd(acc + 3 * p + 2, ec.z);
                    }
                }
            }
        }
    }
    flush_work<COUNT>(w, work_out);
}

// Visibility bits of the queue entries [begin, end) cleared before a binned shadow launch.
__global__ void k_vis_clear(uint32_t* vis, const uint32_t* begin_p, const uint32_t* count_p, uint32_t cap) {
    const uint32_t end = min(*count_p, cap);
    const uint32_t begin = begin_p ? min(*begin_p, end) : 0u;
    const uint32_t w1 = (end + 31u) >> 5;
    for (uint32_t w = (begin >> 5) + blockIdx.x * blockDim.x + threadIdx.x; w < w1; w += gridDim.x * blockDim.x)
        vis[w] = 0u;
}

// The unblocked entries of a binned shadow launch added to their pixels in
// queue order: a block takes 1024 consecutive entries (a few shading waves'
// rays, light-major), sums them per pixel in an LDS hash table and adds each
// pixel once per channel (path-traced frames: ~7 entries per ray).
constexpr int kVisSlots = 2048;
constexpr uint32_t kVisChunk = 1024;
__global__ __launch_bounds__(256) void k_vis_resolve(ShadowQ s, const uint32_t* vis, const uint32_t* begin_p,
                                                     const uint32_t* count_p, uint32_t cap, float* acc) {
    __shared__ uint32_t key[kVisSlots];
    __shared__ float val[3][kVisSlots];
    const uint32_t end = min(*count_p, cap);
    const uint32_t begin = begin_p ? min(*begin_p, end) : 0u;
    for (uint32_t b = begin + blockIdx.x * kVisChunk; b < end; b += gridDim.x * kVisChunk) {   // block-uniform
        for (int k = threadIdx.x; k < kVisSlots; k += blockDim.x) {
            key[k] = kDeadRay;
            val[0][k] = val[1][k] = val[2][k] = 0.0f;
        }
        __syncthreads();
        for (uint32_t i = b + threadIdx.x; i < min(b + kVisChunk, end); i += blockDim.x) {
            if (!((vis[i >> 5] >> (i & 31u)) & 1u)) continue;
            const float4 ec = s.c[i];
            const uint32_t p = (uint32_t)as_int_f(ec.w);
            uint32_t h = (p * 2654435761u) >> 21;   // 11 bits: a slot of the table
            for (;;) {   // at most 1024 keys in 2048 slots: a free or matching slot is always found
                const uint32_t old = atomicCAS(&key[h], kDeadRay, p);
                if (old == kDeadRay || old == p) break;
                h = (h + 1u) & (kVisSlots - 1u);
            }
            atomicAdd(&val[0][h], ec.x);
            atomicAdd(&val[1][h], ec.y);
            atomicAdd(&val[2][h], ec.z);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < kVisSlots; k += blockDim.x) {
            const uint32_t p = key[k];
            if (p == kDeadRay) continue;
            atomicAdd(acc + 3 * p + 0, val[0][k]);
            atomicAdd(acc + 3 * p + 1, val[1][k]);
            atomicAdd(acc + 3 * p + 2, val[2][k]);
        }
        __syncthreads();
    }
}

// Binning of the deferred shadow queue (a counting sort by key, keys < nb):
// k_bin_count adds per-bin counts, k_bin_scan turns them into first slots,
// k_bin_scatter writes every entry's index into its bin's range of perm.
// Blocks work on chunks of kBinChunk entries with a histogram in LDS, so the
// global atomics are per (chunk, bin), not per entry.  Order inside a bin is
// arbitrary.
constexpr int kBinMax = 4096;
constexpr uint32_t kBinChunk = 16384;
constexpr int kBinBlocks = 4096;   // binning grid: 16 blocks per CU, one chunk each up to 64M entries

__global__ __launch_bounds__(256) void k_bin_count(const uint32_t* key, const uint32_t* begin_p,
                                                   const uint32_t* count_p, uint32_t cap, uint32_t* hist, int nb) {
    __shared__ uint32_t h[kBinMax];
    const uint32_t count = min(*count_p, cap);
    const uint32_t begin = begin_p ? min(*begin_p, count) : 0u;
    for (uint32_t c0 = begin + blockIdx.x * kBinChunk; c0 < count; c0 += gridDim.x * kBinChunk) {   // block-uniform
        for (int b = threadIdx.x; b < nb; b += blockDim.x) h[b] = 0u;
        __syncthreads();
        const uint32_t c1 = min(c0 + kBinChunk, count);
        for (uint32_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) atomicAdd(&h[key[i]], 1u);
        __syncthreads();
        for (int b = threadIdx.x; b < nb; b += blockDim.x)
            if (h[b]) atomicAdd(hist + b, h[b]);
        __syncthreads();
    }
}

// one block of 1024 threads: exclusive scan of hist[0, nb) into first[0, nb)
__global__ __launch_bounds__(1024) void k_bin_scan(const uint32_t* hist, uint32_t* first, int nb) {
    __shared__ uint32_t part[1024];
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per, b1 = min(b0 + per, nb);
    uint32_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += hist[b];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // Hillis-Steele inclusive scan
        const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (int b = b0; b < b1; ++b) {
        first[b] = run;
        run += hist[b];
    }
}

__global__ __launch_bounds__(256) void k_bin_scatter(const uint32_t* key, const uint32_t* begin_p,
                                                     const uint32_t* count_p, uint32_t cap, uint32_t* first,
                                                     uint32_t* perm, int nb) {
    __shared__ uint32_t h[kBinMax];
    const uint32_t count = min(*count_p, cap);
    const uint32_t begin = begin_p ? min(*begin_p, count) : 0u;
    for (uint32_t c0 = begin + blockIdx.x * kBinChunk; c0 < count; c0 += gridDim.x * kBinChunk) {   // block-uniform
        for (int b = threadIdx.x; b < nb; b += blockDim.x) h[b] = 0u;
        __syncthreads();
        const uint32_t c1 = min(c0 + kBinChunk, count);
        for (uint32_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) atomicAdd(&h[key[i]], 1u);
        __syncthreads();
        for (int b = threadIdx.x; b < nb; b += blockDim.x)
            if (h[b]) h[b] = atomicAdd(first + b, h[b]);   // this chunk's range inside the bin
        __syncthreads();
        for (uint32_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) perm[atomicAdd(&h[key[i]], 1u)] = i;
        __syncthreads();
    }
}

// x^n for a non-negative integer n by repeated squaring; other exponents use powf.
__device__ __forceinline__ float pow_spec(float x, float n) {
    if (n == floorf(n) && n <= 4096.0f) {
        int e = (int)n;
        float r = 1.0f, b = x;
        while (e) {
            if (e & 1) r *= b;
            b *= b;
            e >>= 1;
        }
        return r;
    }
    return powf(x, n);
}

// Block-wide reservation: each wave passes its total, one atomic per block and
// queue; returns the wave's base slot.  All threads of the block must call.
__device__ __forceinline__ uint32_t block_reserve(uint32_t wave_total, uint32_t* tail, uint32_t* lds4,
                                                  uint32_t* also = nullptr) {
    const uint32_t wave = threadIdx.x >> 6;
    if (lane_id() == 0) lds4[wave] = wave_total;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t0 = lds4[0], t1 = lds4[1], t2 = lds4[2], t3 = lds4[3];
        const uint32_t tot = t0 + t1 + t2 + t3;
        const uint32_t base = tot ? atomicAdd(tail, tot) : 0u;
        if (tot && also) atomicAdd(also, tot);   // a second count (per-depth statistics)
        lds4[0] = base;
        lds4[1] = base + t0;
        lds4[2] = base + t0 + t1;
        lds4[3] = base + t0 + t1 + t2;
    }
    __syncthreads();
    const uint32_t r = lds4[wave];
    __syncthreads();
    return r;
}

// Two reservations in one block-wide pass (the shadow rays and the next
// depth's rays of a shading block).  lds8: 8 words.  All threads must call.
__device__ __forceinline__ void block_reserve2(uint32_t tot_a, uint32_t* tail_a, uint32_t* also_a, uint32_t tot_b,
                                               uint32_t* tail_b, uint32_t* lds8, uint32_t& base_a,
                                               uint32_t& base_b) {
    const uint32_t wave = threadIdx.x >> 6;
    if (lane_id() == 0) {
        lds8[wave] = tot_a;
        lds8[4 + wave] = tot_b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 2; ++k) {
            uint32_t* v = lds8 + 4 * k;
            const uint32_t t0 = v[0], t1 = v[1], t2 = v[2], t3 = v[3];
            const uint32_t tot = t0 + t1 + t2 + t3;
            const uint32_t base = tot ? atomicAdd(k ? tail_b : tail_a, tot) : 0u;
            if (tot && !k && also_a) atomicAdd(also_a, tot);   // a second count (per-depth statistics)
            v[0] = base;
            v[1] = base + t0;
            v[2] = base + t0 + t1;
            v[3] = base + t0 + t1 + t2;
        }
    }
    __syncthreads();
    base_a = lds8[wave];
    base_b = lds8[4 + wave];
    __syncthreads();
}

struct LightTerm {
    float cr, cg, cb;
    bool emit;
};

// Point of light l for pass (frame, sample s): the light's position, or for an
// area light one point of its parallelogram or ellipse from the camera-jitter
// hash with the pixel slot 0xFFFFFFFF - l (the same for every pixel of the
// pass), computed in FP64 and rounded once.
__device__ __forceinline__ V3 light_point(const DevLight& L, uint64_t seed, uint32_t frame, uint32_t s, int l) {
    const int shape = (int)L.pos.w;
    if (shape == RT_LIGHT_POINT) return xyz(L.pos);
    const double a = jitter01(seed, frame, 0xFFFFFFFFu - (uint32_t)l, s, 0);
    const double b = jitter01(seed, frame, 0xFFFFFFFFu - (uint32_t)l, s, 1);
    double cu = a, cv = b;
    if (shape == RT_LIGHT_DISK) {
        const double r = sqrt(a);
        double sn, cs;
        sincos(2.0 * M_PI * b, &sn, &cs);
        cu = r * cs;
        cv = r * sn;
    }
    return v3((float)((double)L.pos.x + cu * (double)L.u.x + cv * (double)L.v.x),
              (float)((double)L.pos.y + cu * (double)L.u.y + cv * (double)L.v.y),
              (float)((double)L.pos.z + cu * (double)L.u.z + cv * (double)L.v.z));
}

// Sample points of every light for every pass of a frame: out[s * n + l].
// The frame number is read on the device (a replayed graph sees the new one).
__global__ void k_light_points(const DevLight* lights, int n, int spp, uint64_t seed, const uint32_t* frame_p,
                               float4* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * spp) return;
    const V3 p = light_point(lights[i % n], seed, *frame_p, (uint32_t)(i / n), i % n);
    out[i] = make_float4(p.x, p.y, p.z, 0.0f);
}

// Batched frames: every scene's light-point table, scenes found by binary
// search over their first entries (everything read from the device table).
__global__ void k_light_points_batch(const BatchScene* tab, int n_scenes, uint32_t total) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int lo = 0, hi = n_scenes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].lpt_first <= e) lo = mid;
        else hi = mid - 1;
    }
    const BatchScene& B = tab[lo];
    const uint32_t i = e - B.lpt_first;
    if (i >= B.lpt_count) return;
    const int n = B.sc.n_lights;
    const V3 p = light_point(B.sc.lights[i % n], B.shc.seed, B.cam.frame, i / n, (int)(i % n));
    const_cast<float4*>(B.shc.light_pts)[i] = make_float4(p.x, p.y, p.z, 0.0f);
}

// Light l's point for pass s: from the frame's table, or the light itself.
__device__ __forceinline__ V3 light_at(const DevScene& S, const ShadeConst& C, uint32_t s, int l) {
    return C.light_pts ? xyz(C.light_pts[(size_t)s * S.n_lights + l]) : xyz(S.lights[l].pos);
}

// Phong light term (without visibility) of a light of intensity I at point lp,
// seen from x with facing normal nf.
__device__ __forceinline__ LightTerm light_term(V3 lp, float4 intensity, V3 x, V3 nf, V3 d, V3 alb, float kd,
                                                float ks, float shin) {
    LightTerm t{0.0f, 0.0f, 0.0f, false};
    V3 lv = lp - x;
    lv = lv * (1.0f / sqrtf(dot(lv, lv)));
    const float ndl = dot(nf, lv);
    if (ndl <= 0.0f) return t;
    const V3 rr = (2.0f * ndl) * nf - lv;
    const float rv = fmaxf(0.0f, -dot(rr, d));
    const float spec = ks * pow_spec(rv, shin);
    const V3 I = xyz(intensity);
    t.cr = I.x * (kd * alb.x * ndl + spec);
    t.cg = I.y * (kd * alb.y * ndl + spec);
    t.cb = I.z * (kd * alb.z * ndl + spec);
    t.emit = fmaxf(t.cr, fmaxf(t.cg, t.cb)) > 0.0f;
    return t;
}

__device__ __forceinline__ uint32_t bin_axis(float x, float lo, float inv, int c) {
    const float f = fminf(fmaxf((x - lo) * inv, 0.0f), (float)(c - 1));   // NaN -> 0
    return (uint32_t)f;
}

// Shadow-queue records are written during the bounces and read only by the
// shadow launch at the end of the frame: non-temporal stores keep them from
// evicting the BVH node and ray-queue lines the bounces re-read from the L2.
__device__ __forceinline__ void store_stream(float4* p, float4 v) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    const f4v x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<f4v*>(p));
}

template <bool STREAM>
__device__ __forceinline__ void write_shadow(const ShadowQ& sq, uint32_t slot, uint32_t cap, uint32_t* ctr, V3 xs,
                                             V3 lp, V3 w, const LightTerm& lt, uint32_t pix, uint32_t sid,
                                             const ShadeConst& C, int l) {
    if (slot >= cap) {
        atomicOr(ctr + kCtrStatus, 2u);
        return;
    }
    // The segment is traced from the light towards the offset surface point: the rays of one light in a
    // wave then leave from one point and share their first node visits (occlusion is symmetric).
    V3 sd = xs - lp;
    const float dist = sqrtf(dot(sd, sd));
    sd = sd * (1.0f / dist);
    const float4 a = make_float4(lp.x, lp.y, lp.z, dist), b = make_float4(sd.x, sd.y, sd.z, as_float_i((int)sid)),
                 c = make_float4(w.x * lt.cr, w.y * lt.cg, w.z * lt.cb, as_float_i((int)pix));
    if (STREAM) {
        store_stream(sq.a + slot, a);
        store_stream(sq.b + slot, b);
        store_stream(sq.c + slot, c);
    } else {
        sq.a[slot] = a;
        sq.b[slot] = b;
        sq.c[slot] = c;
    }
    if (sq.key) {
        const int c = C.bin_c;
        const uint32_t cell = bin_axis(xs.x, C.bin_lo[0], C.bin_inv[0], c) +
                              (uint32_t)c * (bin_axis(xs.y, C.bin_lo[1], C.bin_inv[1], c) +
                                             (uint32_t)c * bin_axis(xs.z, C.bin_lo[2], C.bin_inv[2], c));
        __builtin_nontemporal_store((uint32_t)(l & 31) * (uint32_t)(c * c * c) + cell, sq.key + slot);
    }
}

// Shading of one depth: Phong local terms (ambient now, light terms deferred to
// the shadow kernel), reflected / refracted rays into the next queue.  Queue
// slots are reserved with one atomic per block and queue; shadow rays are laid
// out light-major inside each wave (consecutive entries go to the same light)
// so the shadow kernel's waves traverse coherently.
// GI: compiled with the path-tracing branch (taken where the scene's ShadeConst has gi set).
// Six waves per SIMD: the register count lands just above the 80 that allow them.
template <bool BATCH, bool GI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_shade(DevScene sc, ShadeConst c0, const BatchScene* tab, RayQ qin, HitQ hit,
                                               uint32_t* ctr, int depth, RayQ qout, ShadowQ sq, float* acc) {
    __shared__ uint32_t lds_res[8];
    __shared__ float lds_add[3][256];   // depth 0: the block's background / ambient terms ...
    __shared__ uint32_t lds_pix[256];   // ... and their pixels
    const uint32_t qcap = c0.qcap, scap = c0.scap;
    const uint32_t count = min(ctr[kCtrRays + depth], qcap);
    const uint32_t stride = gridDim.x * blockDim.x;
    const bool light_major = !BATCH && sc.n_lights <= 32;
    const bool sum0 = !BATCH && depth == 0 && c0.sum_depth0;
    for (uint32_t bb = blockIdx.x * blockDim.x; bb < count; bb += stride) {   // block-uniform loop
        const uint32_t i = bb + threadIdx.x;
        bool active = i < count;
        int prim = -1;
        uint32_t pix = 0, meta = 0;
        V3 o = v3(0, 0, 0), d = v3(0, 0, 1), w = v3(0, 0, 0);
        float t = 0.0f;
        float4 ra = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (active) {
            ra = BATCH ? qin.a[i] : load_stream(qin.a + i);
            pix = (uint32_t)as_int_f(ra.w);
            active = pix != kDeadRay;
        }
        if (active) {
            prim = BATCH ? hit.prim[i] : __builtin_nontemporal_load(hit.prim + i);
            t = BATCH ? hit.t[i] : __builtin_nontemporal_load(hit.t + i);
            const float4 rb = BATCH ? qin.b[i] : load_stream(qin.b + i), rc = BATCH ? qin.c[i] : load_stream(qin.c + i);
            meta = (uint32_t)as_int_f(rb.w);
            o = v3(ra.x, ra.y, ra.z);
            d = v3(rb.x, rb.y, rb.z);
            w = v3(rc.x, rc.y, rc.z);
        }
        const uint32_t sid = BATCH ? (meta >> 20) : 0u;
        const DevScene& S = scene_of<BATCH>(sc, tab, sid);
        const ShadeConst& C = shade_of<BATCH>(c0, tab, sid);
        const uint32_t smp = (meta >> 4) & 0xFFFFu;   // the ray's pass: selects the area lights' points
        if (active && depth == 0 && C.out_ids) {
            int oid = -1;
            if (prim >= S.n_bvh) oid = prim;
            else if (prim >= 0) oid = as_int_f(S.prims[3 * prim].w);
            const uint32_t local = pix - C.acc_off;
            C.out_ids[C.per_sample ? (size_t)local : (size_t)local * C.spp + ((meta >> 4) & 0xFFFFu)] = oid;
        }
        const bool shade = active && prim >= 0;
        V3 add = v3(0.0f, 0.0f, 0.0f);   // background (miss) or ambient (hit) term of this ray
        bool has_add = false;
        if (active && prim < 0) {
            add = v3(w.x * C.bg[0], w.y * C.bg[1], w.z * C.bg[2]);
            has_add = true;
        }
        // hit point, geometric normal, material
        V3 x = v3(0, 0, 0), ng = v3(0, 0, 1);
        int mat = 0;
        if (shade) {
            x = v3(fmaf(t, d.x, o.x), fmaf(t, d.y, o.y), fmaf(t, d.z, o.z));
            if (prim >= S.n_bvh) {
                const float4 pl = S.planes[prim - S.n_bvh];
                ng = xyz(pl);
                mat = S.plane_mat[prim - S.n_bvh];
            } else {
                // a triangle's normal record carries its material: one read; a sphere's holds ~material
                const float4 nr = S.normals[prim];
                const int code = as_int_f(nr.w);
                if (code >= 0) {
                    ng = xyz(nr);
                    mat = code;
                } else {
                    const float4 p0 = S.prims[3 * prim];
                    const float4 p1 = S.prims[3 * prim + 1];
                    mat = ~code;
                    ng = (x - xyz(p0)) * p1.z;
                    ng = ng * (1.0f / sqrtf(dot(ng, ng)));
                }
            }
        }
        const float dn = dot(d, ng);
        const bool entering = dn < 0.0f;
        const V3 nf = entering ? ng : -ng;
        const DevMaterial M = S.mats[mat];
        const V3 alb = xyz(M.a);
        const float ka = M.a.w, kd = M.b.x, ks = M.b.y, shin = M.b.z, kr = M.b.w, ior = M.c.x;
        const int type = (int)M.c.y;
        const float eps_s = C.eps * fmaxf(1.0f, maxabs(x));
        const V3 xs = x + eps_s * nf;
        if (shade && ka > 0.0f) {
            add = v3(w.x * ka * alb.x, w.y * ka * alb.y, w.z * ka * alb.z);
            has_add = true;
        }
        if (sum0) {
            add_block_terms(acc, has_add, pix, add, lds_add, lds_pix);
        } else if (has_add) {
            atomicAdd(acc + 3 * pix + 0, add.x);
            atomicAdd(acc + 3 * pix + 1, add.y);
            atomicAdd(acc + 3 * pix + 2, add.z);
        }
        // a block whose rays all missed spawns nothing: skip the reservations and their barriers
        if (!__syncthreads_or(shade ? 1 : 0)) continue;
        // ---- shadow rays: decide per light, reserve, then write
        uint32_t emit_mask = 0, n_sh = 0;
        if (shade) {
            for (int l = 0; l < S.n_lights; ++l) {
                const LightTerm lt = light_term(light_at(S, C, smp, l), S.lights[l].intensity, x, nf, d, alb, kd, ks,
                                                shin);
                if (lt.emit) {
                    n_sh++;
                    if (l < 32) emit_mask |= 1u << l;
                }
            }
        }
        // ---- secondary rays
        bool want_r = false, want_t = false;
        float wr_s = 0.0f, wt_s = 0.0f;   // Whitted branch weights (scalars)
        V3 dr = v3(0, 0, 0), dt = v3(0, 0, 0);
        const float cosi = entering ? -dn : dn;   // = -d.nf >= 0
        if (shade && depth < C.max_depth) {
            dr = d + (2.0f * cosi) * nf;
            dr = dr * (1.0f / sqrtf(dot(dr, dr)));
            if (type == RT_MAT_DIELECTRIC) {
                const float eta = entering ? 1.0f / ior : ior;
                const float k2 = 1.0f - eta * eta * (1.0f - cosi * cosi);
                const float r0 = ((ior - 1.0f) / (ior + 1.0f)) * ((ior - 1.0f) / (ior + 1.0f));
                float F = 1.0f;
                if (k2 >= 0.0f) {
                    const float ck = sqrtf(k2);
                    const float cc = entering ? cosi : ck;
                    const float om = 1.0f - cc;
                    F = r0 + (1.0f - r0) * (om * om * om * om * om);
                    dt = eta * d + (eta * cosi - ck) * nf;
                    dt = dt * (1.0f / sqrtf(dot(dt, dt)));
                    want_t = true;
                    wt_s = 1.0f - F;
                }
                want_r = true;
                wr_s = F;
            } else if (kr > 0.0f) {
                want_r = true;
                wr_s = kr;
            }
        }
        V3 fr = v3(wr_s, wr_s, wr_s), ft = v3(wt_s, wt_s, wt_s);   // factors of the spawned rays' weights
        if (GI && C.gi && shade && depth < C.max_depth) {
            // path tracing: one branch among diffuse (k_d albedo), reflect and refract, chosen with
            // probability m_x / S (m_x: largest channel of the branch weight), weighted by weight * S / m_x
            const uint32_t frame = BATCH ? tab[sid].cam.frame : ctr[kCtrFrame];
            const uint32_t local = pix - C.acc_off;
            const uint32_t pixel = C.per_sample ? local / (uint32_t)C.spp : local;
            const float md = kd > 0.0f ? kd * fmaxf(alb.x, fmaxf(alb.y, alb.z)) : 0.0f;
            const float mr = want_r ? wr_s : 0.0f, mt = want_t ? wt_s : 0.0f;
            const float ssum = md + mr + mt;
            int pick = -1;
            if (ssum > 0.0f) {
                const float us = path_rand(C.seed, frame, pixel, smp, (uint32_t)depth, 0u) * ssum;
                float cum = 0.0f;
                int last = -1;
                if (md > 0.0f) {
                    cum += md;
                    last = 0;
                    if (us < cum) pick = 0;
                }
                if (mr > 0.0f) {
                    cum += mr;
                    last = 1;
                    if (pick < 0 && us < cum) pick = 1;
                }
                if (mt > 0.0f) {
                    cum += mt;
                    last = 2;
                    if (pick < 0 && us < cum) pick = 2;
                }
                if (pick < 0) pick = last;
            }
            want_r = pick == 0 || pick == 1;
            want_t = pick == 2;
            fr = v3(ssum, ssum, ssum);
            ft = fr;
            if (pick == 0) {
                // cosine-weighted: N_f plus a point uniform on the unit sphere, normalized
                const float z = 1.0f - 2.0f * path_rand(C.seed, frame, pixel, smp, (uint32_t)depth, 1u);
                const float phi = 6.28318530717958647692f * path_rand(C.seed, frame, pixel, smp, (uint32_t)depth, 2u);
                const float r = sqrtf(fmaxf(0.0f, 1.0f - z * z));
                float sp, cp;
                sincosf(phi, &sp, &cp);
                const V3 dd = nf + v3(r * cp, r * sp, z);
                const float len = sqrtf(dot(dd, dd));
                want_r = len > 0.0f;
                dr = dd * (1.0f / len);
                const float g = kd * (ssum / md);
                fr = v3(g * alb.x, g * alb.y, g * alb.z);
            }
        }
        // ---- one block-wide reservation for both: shadow rays (deferred: one queue for the shadow rays of
        // every depth, traced once at the end of the pass) and the next depth's rays
        const uint32_t nsec = (want_r ? 1u : 0u) + (want_t ? 1u : 0u);
        uint32_t wave_tot, sec_tot;
        const uint32_t lane_off = wave_scan(n_sh, wave_tot);
        const uint32_t sec_off = wave_scan(nsec, sec_tot);
        uint32_t wave_base, sec_base;
        block_reserve2(wave_tot, C.defer_shadow ? ctr + kCtrShadowAll : ctr + kCtrShadow + depth,
                       C.defer_shadow ? ctr + kCtrShadow + depth : nullptr, sec_tot, ctr + kCtrRays + depth + 1,
                       lds_res, wave_base, sec_base);
        if (light_major) {
            // light-major: for each light, the wave's emitting lanes take consecutive slots
            uint32_t run = wave_base;
            for (int l = 0; l < S.n_lights; ++l) {   // wave-uniform loop
                const bool e = (emit_mask >> l) & 1u;
                const uint64_t bal = __ballot(e);
                if (e) {
                    const uint32_t slot = run + __builtin_amdgcn_mbcnt_hi(
                                                    (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                    const V3 lp = light_at(S, C, smp, l);
                    const LightTerm lt = light_term(lp, S.lights[l].intensity, x, nf, d, alb, kd, ks, shin);
                    write_shadow<!BATCH>(sq, slot, scap, ctr, xs, lp, w, lt, pix, sid, C, l);
                }
                run += (uint32_t)__popcll(bal);
            }
        } else if (n_sh) {
            uint32_t slot = wave_base + lane_off;   // lane-major (more than 32 lights)
            for (int l = 0; l < S.n_lights; ++l) {
                const V3 lp = light_at(S, C, smp, l);
                const LightTerm lt = light_term(lp, S.lights[l].intensity, x, nf, d, alb, kd, ks, shin);
                if (!lt.emit) continue;
                write_shadow<!BATCH>(sq, slot++, scap, ctr, xs, lp, w, lt, pix, sid, C, l);
            }
        }
        uint32_t qslot = sec_base + sec_off;
        const uint32_t meta_next = (meta & ~15u) | (uint32_t)(depth + 1);
        if (want_r) {
            if (qslot < qcap) {
                qout.a[qslot] = make_float4(xs.x, xs.y, xs.z, as_float_i((int)pix));
                qout.b[qslot] = make_float4(dr.x, dr.y, dr.z, as_float_i((int)meta_next));
                qout.c[qslot] = make_float4(w.x * fr.x, w.y * fr.y, w.z * fr.z, 0.0f);
            } else {
                atomicOr(ctr + kCtrStatus, 1u);
            }
            qslot++;
        }
        if (want_t) {
            if (qslot < qcap) {
                const V3 xt = x - eps_s * nf;
                qout.a[qslot] = make_float4(xt.x, xt.y, xt.z, as_float_i((int)pix));
                qout.b[qslot] = make_float4(dt.x, dt.y, dt.z, as_float_i((int)meta_next));
                qout.c[qslot] = make_float4(w.x * ft.x, w.y * ft.y, w.z * ft.z, 0.0f);
            } else {
                atomicOr(ctr + kCtrStatus, 1u);
            }
        }
    }
}

// Batched resolve: each accumulation float goes to its scene's output.
__global__ void k_resolve_batch(const BatchScene* tab, int n_scenes, const float* acc, uint64_t n3) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const uint32_t slot = (uint32_t)(i / 3);
    int lo = 0, hi = n_scenes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].shc.acc_off <= slot) lo = mid;
        else hi = mid - 1;
    }
    const BatchScene& B = tab[lo];
    B.out_rgb[(size_t)(slot - B.shc.acc_off) * 3 + (i - (uint64_t)slot * 3)] = acc[i] * B.inv_spp;
}


// ---------------------------------------------------------------------------
// learned form: radiance cache below depth D_c
// ---------------------------------------------------------------------------
// Feature layout of one cache query (BF16, 64 values): for axis c and
// frequency j, [12 c + 2 j] = sin(2^j pi x~_c), [12 c + 2 j + 1] = cos(...),
// x~ = 2 (x - lo) / (hi - lo) - 1; [36..38] facing normal; [39..41] view
// direction; [42..63] zero.
struct CacheRec {
    uint16_t* feats;     // [cap][64]
    uint32_t* pix;       // [cap] accumulation slot
    float* w;            // [cap][3] throughput
    uint32_t* src;       // [cap] queue index of the ray at the cache depth
    uint32_t cap;
};

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ void write_features(uint16_t* f, V3 x, V3 nf, V3 v, const float* lo, const float* inv_ext) {
    const float xt[3] = {2.0f * (x.x - lo[0]) * inv_ext[0] - 1.0f, 2.0f * (x.y - lo[1]) * inv_ext[1] - 1.0f,
                         2.0f * (x.z - lo[2]) * inv_ext[2] - 1.0f};
    uint16_t tmp[64];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float sc = 1.0f;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            tmp[12 * c + 2 * j] = to_bf16(sinpif(sc * xt[c]));
            tmp[12 * c + 2 * j + 1] = to_bf16(cospif(sc * xt[c]));
            sc *= 2.0f;
        }
    }
    tmp[36] = to_bf16(nf.x);
    tmp[37] = to_bf16(nf.y);
    tmp[38] = to_bf16(nf.z);
    tmp[39] = to_bf16(v.x);
    tmp[40] = to_bf16(v.y);
    tmp[41] = to_bf16(v.z);
#pragma unroll
    for (int k = 42; k < 64; ++k) tmp[k] = 0;
    uint4* dst = reinterpret_cast<uint4*>(f);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        uint4 u;
        u.x = (uint32_t)tmp[8 * q + 0] | ((uint32_t)tmp[8 * q + 1] << 16);
        u.y = (uint32_t)tmp[8 * q + 2] | ((uint32_t)tmp[8 * q + 3] << 16);
        u.z = (uint32_t)tmp[8 * q + 4] | ((uint32_t)tmp[8 * q + 5] << 16);
        u.w = (uint32_t)tmp[8 * q + 6] | ((uint32_t)tmp[8 * q + 7] << 16);
        dst[q] = u;
    }
}

// Shading at the cache depth: misses add the background; hits become cache
// queries (features, accumulation slot, throughput, source ray).
__global__ __launch_bounds__(256) void k_cache_shade(DevScene sc, ShadeConst c, RayQ qin, HitQ hit, uint32_t* ctr,
                                                     int depth, CacheRec rec, float lo0, float lo1, float lo2,
                                                     float ie0, float ie1, float ie2, float* acc) {
    __shared__ uint32_t lds_res[4];
    const uint32_t count = min(ctr[kCtrRays + depth], c.qcap);
    const uint32_t stride = gridDim.x * blockDim.x;
    const float lo[3] = {lo0, lo1, lo2}, ie[3] = {ie0, ie1, ie2};
    for (uint32_t bb = blockIdx.x * blockDim.x; bb < count; bb += stride) {   // block-uniform loop
        const uint32_t i = bb + threadIdx.x;
        bool active = i < count;
        uint32_t pix = 0, meta = 0;
        int prim = -1;
        float4 ra = make_float4(0.0f, 0.0f, 0.0f, 0.0f), rb = ra;
        if (active) {
            ra = qin.a[i];
            pix = (uint32_t)as_int_f(ra.w);
            active = pix != kDeadRay;
        }
        V3 w = v3(0, 0, 0);
        if (active) {
            prim = hit.prim[i];
            rb = qin.b[i];
            meta = (uint32_t)as_int_f(rb.w);
            const float4 rc = qin.c[i];
            w = v3(rc.x, rc.y, rc.z);
            if (depth == 0 && c.out_ids) {
                int oid = -1;
                if (prim >= sc.n_bvh) oid = prim;
                else if (prim >= 0) oid = as_int_f(sc.prims[3 * prim].w);
                c.out_ids[c.per_sample ? (size_t)pix : (size_t)pix * c.spp + ((meta >> 4) & 0xFFFFu)] = oid;
            }
            if (prim < 0) {
                atomicAdd(acc + 3 * pix + 0, w.x * c.bg[0]);
                atomicAdd(acc + 3 * pix + 1, w.y * c.bg[1]);
                atomicAdd(acc + 3 * pix + 2, w.z * c.bg[2]);
            }
        }
        const bool query = active && prim >= 0;
        uint32_t tot;
        const uint32_t off = wave_scan(query ? 1u : 0u, tot);
        const uint32_t slot = block_reserve(tot, ctr + kCtrRec, lds_res) + off;
        if (query) {
            if (slot >= rec.cap) {
                atomicOr(ctr + kCtrStatus, 4u);
                continue;
            }
            const V3 o = v3(ra.x, ra.y, ra.z);
            const V3 d = v3(rb.x, rb.y, rb.z);
            const float t = hit.t[i];
            const V3 x = v3(fmaf(t, d.x, o.x), fmaf(t, d.y, o.y), fmaf(t, d.z, o.z));
            V3 ng;
            if (prim >= sc.n_bvh) {
                ng = xyz(sc.planes[prim - sc.n_bvh]);
            } else {
                const float4 nr = sc.normals[prim];
                if (as_int_f(nr.w) >= 0) {   // a triangle (a sphere's record holds ~material)
                    ng = xyz(nr);
                } else {
                    const float4 p0 = sc.prims[3 * prim];
                    ng = (x - xyz(p0)) * sc.prims[3 * prim + 1].z;
                    ng = ng * (1.0f / sqrtf(dot(ng, ng)));
                }
            }
            const V3 nf = dot(d, ng) < 0.0f ? ng : -ng;
            write_features(rec.feats + (size_t)slot * 64, x, nf, -d, lo, ie);
            rec.pix[slot] = pix;
            rec.w[3 * slot + 0] = w.x;
            rec.w[3 * slot + 1] = w.y;
            rec.w[3 * slot + 2] = w.z;
            rec.src[slot] = i;
        }
    }
}

// Training batch of this frame: n_train = min(queries, train_samples) queries
// chosen on a stratified grid with a per-frame random offset.  Their rays (at
// the cache depth) start the target wavefront; their features and rays are
// kept in the cache state.
__global__ void k_cache_select(const uint32_t* ctr, CacheRec rec, RayQ qsrc, uint32_t train_samples, int depth,
                               RayQ qt, uint32_t* ctr_t, uint32_t* n_train_out, uint16_t* t_feats, float* t_rays,
                               uint32_t* t_pix) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t queries = min(ctr[kCtrRec], rec.cap);
    const uint32_t n_train = min(queries, train_samples);
    if (j == 0) {
        *n_train_out = n_train;
        ctr_t[kCtrRays + depth] = n_train;
    }
    if (j >= n_train) return;
    const uint32_t frame = ctr[kCtrFrame];
    const double u = (double)(pcg_hash(pcg_hash(frame ^ 0x9e3779b9u)) >> 8) * (1.0 / 16777216.0);
    uint32_t src = (uint32_t)(((double)j + u) * (double)queries / (double)n_train);
    src = min(src, queries - 1u);
    const uint32_t i = rec.src[src];
    const float4 sa = qsrc.a[i], sb = qsrc.b[i];
    qt.a[j] = make_float4(sa.x, sa.y, sa.z, as_float_i((int)j));
    qt.b[j] = make_float4(sb.x, sb.y, sb.z, as_float_i(depth));
    qt.c[j] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
    const uint4* fs = reinterpret_cast<const uint4*>(rec.feats + (size_t)src * 64);
    uint4* fd = reinterpret_cast<uint4*>(t_feats + (size_t)j * 64);
    for (int q = 0; q < 8; ++q) fd[q] = fs[q];
    t_rays[6 * j + 0] = sa.x;
    t_rays[6 * j + 1] = sa.y;
    t_rays[6 * j + 2] = sa.z;
    t_rays[6 * j + 3] = sb.x;
    t_rays[6 * j + 4] = sb.y;
    t_rays[6 * j + 5] = sb.z;
    t_pix[j] = rec.pix[src];
}

// Cache-state counter words: [0] Adam steps, [1] training samples of the last
// frame, [2 .. 18) the last frame's per-step loss sums, [kCacheHealth] health
// bits (bit 0 a non-finite loss sum, bit 1 a non-finite master weight or Adam
// moment after training, bit 2 a non-finite BF16 weight at the start of a
// frame).  Bits stay set until the state is initialised again.
constexpr int kCacheHealth = 18;

// The learned form's gate, between the closest hits at the cache depth and
// their shading.  A healthy cache leaves the frame as it is.  An unhealthy one
// (any health bit, or a non-finite BF16 weight now) hands the depth's hits to
// the fallback chain: their count moves from the frame's counters to the
// chain's, so the network sees no query and the plain tracer shades them and
// carries their paths on to the full depth.  One thread per weight; the last
// block to finish (the chain's counters, cleared each frame, collect the
// blocks' findings and count the finished blocks) takes the decision.
constexpr int kCtrGateBad = 100;    // fallback chain's counters: non-finite BF16 weights seen by the gate
constexpr int kCtrGateDone = 101;   // ... and the gate's finished blocks
__global__ __launch_bounds__(256) void k_cache_gate(const uint16_t* wb, int n, uint32_t* health, uint32_t* ctr,
                                                    uint32_t* ctr_fb, int depth, rt_stats* st) {
    __shared__ uint32_t last;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool bad = i < n && (wb[i] & 0x7F80u) == 0x7F80u;   // BF16 exponent all ones: Inf or NaN
    if (__any(bad) && lane_id() == 0) atomicOr(ctr_fb + kCtrGateBad, 4u);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(ctr_fb + kCtrGateDone, 1u) == gridDim.x - 1 ? 1u : 0u;
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    __threadfence();
    const uint32_t seen = atomicOr(ctr_fb + kCtrGateBad, 0u);
    uint32_t h = *health;
    if (seen) {
        h |= seen;
        *health = h;
    }
    if (h == 0u) return;
    ctr_fb[kCtrRays + depth] = ctr[kCtrRays + depth];
    ctr[kCtrRays + depth] = 0u;
    if (st) atomicOr(&st->status, (uint32_t)RT_STATUS_CACHE_FALLBACK);
}

__global__ void k_resolve(const float* acc, float* out, int64_t n3, float inv_spp, const uint32_t* accum) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) out[i] = acc[i] * (inv_spp / (float)(*accum + 1u));
}

// clears the accumulator unless the frame adds to earlier ones (progressive mode)
__global__ void k_clear_acc(float* acc, int64_t n, const uint32_t* accum) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && *accum == 0u) acc[i] = 0.0f;
}

// fold a pass's queue counters into the caller's statistics
// part 0: a frame's pass; 1: a learned-form frame (also its network queries);
// 2: the rays traced for training targets (kept apart from the image's rays);
// 3: the learned form's fallback chain (rays of the frame's own pass)
__global__ void k_stats(const uint32_t* ctr, rt_stats* st, int max_depth, int part) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (!st) return;
    st->status |= ctr[kCtrStatus];
    if (part == 2) {
        uint64_t r = 0, s = 0;
        for (int k = 0; k <= max_depth && k < RT_STATS_MAX_DEPTH; ++k) {
            r += ctr[kCtrRays + k];
            s += ctr[kCtrShadow + k];
        }
        st->target_rays += r;
        st->target_shadow += s;
        return;
    }
    if (part != 3) st->passes += 1;   // part 3: the learned form's fallback chain (depths of the same pass)
    for (int k = 0; k <= max_depth && k < RT_STATS_MAX_DEPTH; ++k) {
        st->rays[k] += (uint64_t)ctr[kCtrRays + k] - (k == 0 ? (uint64_t)ctr[kCtrDead] : 0ull);
        st->shadow[k] += (uint64_t)ctr[kCtrShadow + k];
    }
    if (part == 1) st->cache_queries += ctr[kCtrRec];
}


// Surface coordinates of a closest hit (rt_intersect's uv output).  Triangle:
// the barycentric weights of its second and third vertex, V/det and W/det of
// the watertight test's edge functions (U goes with the first vertex), so
// that the hit point is (1-u-v) v0 + u v1 + v v2.  Sphere: the outward
// normal n = (x - c)/r at x = o + t d in spherical coordinates, u =
// (atan2(n_z, n_x) + pi) / (2 pi), v = acos(n_y) / pi.  Planes and misses: 0.
__device__ float2 hit_uv(const DevScene& sc, const TRay& r, const Hit& h) {
#pragma clang fp contract(off)
    if (h.prim < 0 || h.prim >= sc.n_bvh) return make_float2(0.0f, 0.0f);
    const float4 p0 = sc.prims[3 * h.prim], p1 = sc.prims[3 * h.prim + 1];
    if (h.id < sc.n_spheres) {
        const V3 x = r.o + h.t * r.d;
        const V3 n = (x - xyz(p0)) * p1.z;
        const float ny = fminf(1.0f, fmaxf(-1.0f, n.y));
        const float kPi = 3.14159265358979f;
        return make_float2((atan2f(n.z, n.x) + kPi) / (2.0f * kPi), acosf(ny) / kPi);
    }
    const float4 p2 = sc.prims[3 * h.prim + 2];
    const V3 A = xyz(p0) - r.o, B = xyz(p1) - r.o, C = xyz(p2) - r.o;
    const float Az = sel(A, r.kz), Bz = sel(B, r.kz), Cz = sel(C, r.kz);
    const float Ax = sel(A, r.kx) - r.sx * Az, Ay = sel(A, r.ky) - r.sy * Az;
    const float Bx = sel(B, r.kx) - r.sx * Bz, By = sel(B, r.ky) - r.sy * Bz;
    const float Cx = sel(C, r.kx) - r.sx * Cz, Cy = sel(C, r.ky) - r.sy * Cz;
    const float U = Cx * By - Cy * Bx, V = Ax * Cy - Ay * Cx, W = Bx * Ay - By * Ax;
    const float det = U + V + W;
    if (det == 0.0f) return make_float2(0.0f, 0.0f);
    return make_float2(V / det, W / det);
}

// Persistent kernels over caller rays (rt_intersect / rt_occluded): same traversal.
template <bool ANY>
__global__ __launch_bounds__(256) void k_trace_rays(DevScene sc, const float* rays, int64_t n, float* t_out,
                                                    int32_t* id_out, float2* uv_out, uint8_t* occ_out,
                                                    uint32_t* cursor) {
    extern __shared__ int32_t smem[];
    LdsStack stk = lds_stack(smem, sc.stack_size);
    Work w{0, 0, 0};
    for (;;) {
        uint32_t base = 0;
        if (lane_id() == 0) base = atomicAdd(cursor, 64u);
        base = __shfl(base, 0, 64);
        if ((int64_t)base >= n) break;
        const int64_t i = (int64_t)base + lane_id();
        if (i < n) {
            const float* R = rays + 8 * i;
            float tmax = R[7];
            if (!(tmax > 0.0f)) tmax = INFINITY;
            const TRay r = make_tray(v3(R[0], R[1], R[2]), v3(R[3], R[4], R[5]));
            const Hit h = traverse<ANY, false>(sc, r, tmax, stk, w);
            if (ANY) {
                occ_out[i] = h.prim >= 0 ? 1 : 0;
            } else {
                t_out[i] = h.prim >= 0 ? h.t : INFINITY;
                id_out[i] = h.prim >= 0 ? h.id : -1;
                if (uv_out) uv_out[i] = hit_uv(sc, r, h);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// host side: device properties, occupancy, workspace plan
// ---------------------------------------------------------------------------
struct DevInfo {
    int cus = 0;
    int max_lds = 0;
};

static rt_status device_info(DevInfo& out) {
    static std::mutex mu;
    static std::map<int, DevInfo> cache;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) {
        out = it->second;
        return RT_OK;
    }
    hipDeviceProp_t p;
    HIP_TRY(hipGetDeviceProperties(&p, dev));
    DevInfo d;
    d.cus = p.multiProcessorCount;
    d.max_lds = (int)p.sharedMemPerBlock;
    cache[dev] = d;
    out = d;
    return RT_OK;
}

// blocks of 256 threads for a persistent traversal kernel: fill every CU to
// the occupancy its LDS stack and registers allow
template <class K>
static rt_status persistent_grid(K kernel, size_t lds, int& blocks) {
    DevInfo di;
    rt_status st = device_info(di);
    if (st != RT_OK) return st;
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, lds));
    blocks = std::max(1, per_cu) * std::max(1, di.cus);
    return RT_OK;
}

struct Plan {
    int64_t npix = 0;
    int64_t nacc = 0;        // accumulation slots: pixels, or pixels * spp per sample
    int spp_pass = 1, passes = 1;
    int64_t n_primary = 0;   // rays of a full pass
    uint32_t qcap = 0, scap = 0;
    size_t off_ctr = 0, off_acc = 0, off_q[2] = {0, 0}, off_hit = 0, off_s = 0, off_s2 = 0, off_bins = 0,
           off_lpts = 0, off_stack = 0, stack_bytes = 0, total = 0;
};

// persistent traversal grids are capped at this many threads; each owns a
// column of the stack overflow region
constexpr uint32_t kMaxPersistentThreads = 1u << 20;

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
// the ray and shadow queues: three arrays of 16-byte records
static size_t shadow_queue_bytes(uint32_t cap) { return 3 * a256(16 * (size_t)cap); }
static size_t ray_queue_bytes(uint32_t cap) { return 3 * a256(16 * (size_t)cap); }

static bool make_plan(const SceneHost& s, const rt_camera& cam, const rt_params& p, Plan& pl, std::string& why,
                      bool bin_space = true) {
    if (cam.width <= 0 || cam.height <= 0) {
        why = "camera width and height must be > 0";
        return false;
    }
    if (p.spp < 1 || p.spp > 65535) {
        why = "spp must be in [1, 65535]";
        return false;
    }
    if (p.max_depth < 0 || p.max_depth > RT_STATS_MAX_DEPTH - 2) {
        why = "max_depth must be in [0, 14]";
        return false;
    }
    if (!tile_ok(p.tile)) {
        why = "tile must be RT_TILE_8X8, RT_TILE_16X4, RT_TILE_32X2 or RT_TILE_4X16";
        return false;
    }
    pl.npix = (int64_t)cam.width * cam.height;
    if (pl.npix > ((int64_t)1 << 31)) {
        why = "too many pixels";
        return false;
    }
    // Path tracing (RT_FLAG_GI) continues a path with at most one ray, so a depth's queue never holds more
    // than the pass's primary rays, and the deferred shadow queue at most (max_depth + 1) x lights per
    // primary ray: exact capacities.  Whitted trees branch; their queues are sized by queue_factor.
    const bool gi = (p.flags & RT_FLAG_GI) != 0;
    const int64_t n_lights = std::max(1, s.n_lights);
    const int64_t target = 32 << 20;   // primary rays per pass when chosen automatically
    const int64_t shadow_target = 512 << 20;   // path tracing: deferred shadow entries per pass, likewise
    int64_t auto_spp = std::min<int64_t>(p.spp, target / pl.npix);
    if (gi) auto_spp = std::min<int64_t>(auto_spp, shadow_target / (pl.npix * (p.max_depth + 1) * n_lights));
    int spp_pass = p.samples_per_pass > 0 ? std::min(p.samples_per_pass, p.spp) : (int)std::max<int64_t>(1, auto_spp);
    pl.spp_pass = spp_pass;
    pl.passes = (p.spp + spp_pass - 1) / spp_pass;
    // ray slots of a full pass: every pixel tile is padded to 64 slots
    pl.n_primary = tiles_x_of(cam.width, p.tile) * tiles_y_of(cam.height, p.tile) * 64 * spp_pass;
    const double qf = p.queue_factor > 0.0f ? std::max(1.0f, p.queue_factor) : (gi ? 1.0 : 2.0);
    const double qcap = std::ceil(pl.n_primary * qf);
    const double scap = gi ? (double)pl.n_primary * (p.max_depth + 1) * n_lights : qcap * n_lights;
    if (qcap > 4.0e9 || scap > 4.0e9) {
        why = "queue capacity exceeds 2^32; lower samples_per_pass or queue_factor";
        return false;
    }
    pl.qcap = (uint32_t)qcap;
    pl.scap = (uint32_t)scap;
    size_t off = 0;
    pl.off_ctr = off;
    off = a256(off + 4 * kCtrTotal);
    pl.nacc = (p.flags & RT_FLAG_PER_SAMPLE) ? pl.npix * p.spp : pl.npix;
    if (pl.nacc >= ((int64_t)1 << 32)) {
        why = "too many accumulation slots (pixels x spp) for per-sample output";
        return false;
    }
    pl.off_acc = off;
    off = a256(off + 12 * (size_t)pl.nacc);
    for (int b = 0; b < 2; ++b) {
        pl.off_q[b] = off;
        off = a256(off + ray_queue_bytes(pl.qcap));
    }
    pl.off_hit = off;
    off = a256(off + 2 * 4 * (size_t)pl.qcap + 2 * 256);
    pl.off_s = off;
    off = a256(off + shadow_queue_bytes(pl.scap));
    // plain frames bin their deferred shadow queue: a key and an order slot per entry
    pl.off_s2 = pl.off_s;
    if (bin_space) {
        pl.off_s2 = off;
        off = a256(off + 2 * a256(4 * (size_t)pl.scap));
    }
    pl.off_bins = off;   // per-bin counts and first slots of the deferred shadow queue
    off = a256(off + 2 * 4 * (size_t)kBinMax);
    pl.off_lpts = off;   // area lights: sample point of every light for every pass of the frame
    if (s.area_lights) off = a256(off + 16 * (size_t)p.spp * (size_t)std::max(1, s.n_lights));
    pl.off_stack = off;   // overflow stacks: closest-hit and shadow traversals
    pl.stack_bytes = a256(4 * (size_t)kMaxPersistentThreads * std::max(0, s.stack_size - kSplitLds));
    off += 2 * pl.stack_bytes;
    pl.total = off;
    return true;
}

static RayQ ray_queue(uint8_t* base, uint32_t cap) {
    const size_t stride = a256(16 * (size_t)cap);
    return RayQ{reinterpret_cast<float4*>(base), reinterpret_cast<float4*>(base + stride),
                reinterpret_cast<float4*>(base + 2 * stride)};
}

static ShadowQ shadow_queue(uint8_t* base, uint32_t cap) {
    const size_t stride = a256(16 * (size_t)cap);
    return ShadowQ{reinterpret_cast<float4*>(base), reinterpret_cast<float4*>(base + stride),
                   reinterpret_cast<float4*>(base + 2 * stride), nullptr};
}

static HitQ hit_queue(uint8_t* base, uint32_t cap) {
    const size_t stride = a256(4 * (size_t)cap);
    return HitQ{reinterpret_cast<float*>(base), reinterpret_cast<int*>(base + stride)};
}

static void camera_consts(const rt_camera& cam, const rt_params& p, CamConst& c) {
    double f[3], r[3], u[3];
    for (int i = 0; i < 3; ++i) f[i] = (double)cam.look_at[i] - cam.eye[i];
    double n = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (double& x : f) x /= n;
    const double up[3] = {cam.up[0], cam.up[1], cam.up[2]};
    r[0] = up[1] * f[2] - up[2] * f[1];
    r[1] = up[2] * f[0] - up[0] * f[2];
    r[2] = up[0] * f[1] - up[1] * f[0];
    n = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (double& x : r) x /= n;
    u[0] = f[1] * r[2] - f[2] * r[1];
    u[1] = f[2] * r[0] - f[0] * r[2];
    u[2] = f[0] * r[1] - f[1] * r[0];
    for (int i = 0; i < 3; ++i) {
        c.eye[i] = cam.eye[i];
        c.f[i] = f[i];
        c.r[i] = r[i];
        c.u[i] = u[i];
    }
    c.th = std::tan((double)cam.vfov_deg * 0.5 * M_PI / 180.0);
    c.aspect = (double)cam.width / cam.height;
    c.W = cam.width;
    c.H = cam.height;
    c.spp = p.spp;
    c.jitter = p.jitter;
    const int m = (int)std::floor(std::sqrt((double)p.spp) + 0.5);
    c.m = (p.spp > 1 && m * m == p.spp) ? m : 0;
    c.frame = p.frame;
    c.seed = p.seed;
    c.tw_log2 = tile_log2w(p.tile);
}

// ---------------------------------------------------------------------------
// optional per-kernel event timing
// ---------------------------------------------------------------------------
struct EventPair {
    int kind;
    hipEvent_t a, b;
};
static std::mutex g_time_mu;
static std::vector<EventPair> g_pending;
static std::vector<hipEvent_t> g_event_pool;
static double g_time_ms[5] = {0, 0, 0, 0, 0};
static int64_t g_time_n[5] = {0, 0, 0, 0, 0};

static hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event pair around one launch when timing is on.
struct KernelTimer {
    bool on;
    hipStream_t st;
    int kind;
    hipEvent_t a = nullptr;
    KernelTimer(bool on_, hipStream_t s, int k) : on(on_), st(s), kind(k) {
        if (!on) return;
        std::lock_guard<std::mutex> g(g_time_mu);
        a = take_event();
        if (a) (void)hipEventRecord(a, st);
    }
    ~KernelTimer() {
        if (!on || !a) return;
        std::lock_guard<std::mutex> g(g_time_mu);
        hipEvent_t b = take_event();
        if (!b) return;
        (void)hipEventRecord(b, st);
        g_pending.push_back(EventPair{kind, a, b});
    }
};

// ---------------------------------------------------------------------------
// frame launch sequence
// ---------------------------------------------------------------------------
struct FrameArgs {
    DevScene sc;
    CamConst cam;
    ShadeConst shc;
    Plan pl;
    uint8_t* ws;
    rt_stats* stats;
    float* out_rgb;
    int32_t* out_ids;
    bool count_work;
    int spp;
    int gx, gs, shade_blocks;   // grid sizes, computed outside any capture
    int gxd;                    // grid of k_extend_deep
    size_t lds;
    bool time_kernels;
    bool time_shadow = false;   // events around the shadow launches only (RT_FLAG_TIME_SHADOW)
    uint32_t chunk;             // queue entries per fetch of a persistent traversal wave
    int tile;                   // RT_TILE_* of the primary rays
    bool bin_shadows;           // deferred shadow rays are binned before their traversal
};

// Calls f with the scene's node layout as a compile-time constant (the
// single-scene traversal kernels are built for each layout).
template <class F>
static void by_layout(int wide, F&& f) {
    if (wide == 2) f(std::integral_constant<int, 2>());
    else if (wide == 1) f(std::integral_constant<int, 1>());
    else f(std::integral_constant<int, 0>());
}

static rt_status frame_grids(FrameArgs& A) {
    A.lds = 0;   // the split stack's LDS part is static
    rt_status s1 = RT_OK, s2 = RT_OK, s3 = RT_OK;
    by_layout(A.sc.wide, [&](auto L) {
        constexpr int kL = decltype(L)::value;
        s1 = A.count_work ? persistent_grid(k_extend<true, false>, 0, A.gx)
                          : persistent_grid(k_extend<false, false, kL>, 0, A.gx);
        s2 = A.count_work ? persistent_grid(k_shadow<true, false>, 0, A.gs)
                          : persistent_grid(k_shadow<false, false, kL>, 0, A.gs);
        s3 = persistent_grid(k_extend_deep<kL>, 0, A.gxd);
    });
    if (s1 != RT_OK) return s1;
    if (s2 != RT_OK) return s2;
    if (s3 != RT_OK) return s3;
    A.gxd = std::min<int>(A.gxd, (int)(kMaxPersistentThreads / 256));
    A.gxd = (int)std::min<int64_t>(A.gxd, std::max<int64_t>(kXcd, ((int64_t)A.pl.qcap + 255) / 256));
    A.gx = std::min<int>(A.gx, (int)(kMaxPersistentThreads / 256));
    A.gs = std::min<int>(A.gs, (int)(kMaxPersistentThreads / 256));
    // small frames: no more blocks than 256-entry slices of the queue (at least one per XCD), so that a
    // launch does not start and retire thousands of idle waves
    A.gx = (int)std::min<int64_t>(A.gx, std::max<int64_t>(kXcd, ((int64_t)A.pl.qcap + 255) / 256));
    A.gs = (int)std::min<int64_t>(A.gs, std::max<int64_t>(kXcd, ((int64_t)A.pl.scap + 255) / 256));
    DevInfo di;
    s1 = device_info(di);
    if (s1 != RT_OK) return s1;
    A.shade_blocks = (int)std::max<int64_t>(1, std::min<int64_t>((A.pl.qcap + 255) / 256, (int64_t)di.cus * 16));
    return RT_OK;
}

// Shadow traversal of the deferred queue's entries [*begin_p, *end_p) on
// stream `st`: optionally binned first (counting sort into perm), then traced
// by `grid` persistent blocks.
struct ShadowSegment {
    const uint32_t* begin_p;   // NULL: from 0
    const uint32_t* end_p;
    uint32_t cap;              // queue capacity
    uint32_t* cursor;
    uint32_t* perm;            // NULL: queue order
    uint32_t* bins;            // [2 * kBinMax]: counts, then first slots
    int32_t* overflow;
    int grid;
};

// Shadow rays of every depth go to one deferred queue, binned by light and by
// a cell of a grid over the scene bounds (at most 4096 bins).
static void defer_and_bin_shadows(FrameArgs& A, const SceneHost& h) {
    A.shc.defer_shadow = 1;
    A.bin_shadows = true;
    const int L = std::max(1, std::min(h.n_lights, 32));
    A.shc.bin_c = L <= 8 ? 8 : 4;   // L * bin_c^3 <= kBinMax
    for (int k = 0; k < 3; ++k) {
        const float lo = h.info.bounds_lo[k], hi = h.info.bounds_hi[k];
        A.shc.bin_lo[k] = lo;
        A.shc.bin_inv[k] = hi > lo ? (float)A.shc.bin_c / (hi - lo) : 0.0f;
    }
}

// Ray generation of a pass.  In a scene without planes, camera rays that miss
// the root's child boxes are finished at once (background into acc); counting
// frames queue every ray, so their node counts cover all camera rays.
static void launch_raygen(const FrameArgs& A, int s0, int ns, int tiles_x, uint32_t nthreads, const RayQ& q,
                          uint32_t* ctr, uint32_t cap, float* acc, hipStream_t st) {
    const RootMiss rm{acc, A.shc.out_ids, {A.shc.bg[0], A.shc.bg[1], A.shc.bg[2]}};
    const dim3 grid((nthreads + 255) / 256);
    if (!A.count_work && A.sc.n_planes == 0)
        by_layout(A.sc.wide, [&](auto L) {
            hipLaunchKernelGGL(k_raygen<decltype(L)::value>, grid, dim3(256), 0, st, A.cam, s0, ns, tiles_x,
                               nthreads, q, ctr, cap, A.shc.per_sample, A.sc, rm);
        });
    else
        hipLaunchKernelGGL(k_raygen<-1>, grid, dim3(256), 0, st, A.cam, s0, ns, tiles_x, nthreads, q, ctr, cap,
                           A.shc.per_sample, A.sc, rm);
}

static void enqueue_shadow_segment(const FrameArgs& A, const ShadowQ& sq, const ShadowSegment& g, int nb, float* acc,
                                   unsigned long long* swork, hipStream_t st) {
    if (g.perm) {
        hipLaunchKernelGGL(k_zero_u32, dim3((nb + 255) / 256), dim3(256), 0, st, g.bins, nb);
        hipLaunchKernelGGL(k_bin_count, dim3(kBinBlocks), dim3(256), 0, st, sq.key, g.begin_p, g.end_p, g.cap, g.bins, nb);
        hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, g.bins, g.bins + kBinMax, nb);
        hipLaunchKernelGGL(k_bin_scatter, dim3(kBinBlocks), dim3(256), 0, st, sq.key, g.begin_p, g.end_p, g.cap,
                           g.bins + kBinMax, g.perm, nb);
    }
    // binned launches mark unblocked entries in the key array (no longer needed once the order is known)
    uint32_t* vis = g.perm && A.shc.gi ? sq.key : nullptr;   // path-traced frames (many unblocked rays)
    if (vis) hipLaunchKernelGGL(k_vis_clear, dim3(1024), dim3(256), 0, st, vis, g.begin_p, g.end_p, g.cap);
    {
        KernelTimer kt(A.time_kernels || A.time_shadow, st, 2);
        if (A.count_work)
            hipLaunchKernelGGL((k_shadow<true, false>), dim3(g.grid), dim3(256), A.lds, st, A.sc, nullptr, sq,
                               g.end_p, g.cursor, g.cap, A.chunk, acc, g.overflow, swork, g.perm, g.begin_p, vis);
        else
            by_layout(A.sc.wide, [&](auto L) {
                hipLaunchKernelGGL((k_shadow<false, false, decltype(L)::value>), dim3(g.grid), dim3(256), A.lds, st,
                                   A.sc, nullptr, sq, g.end_p, g.cursor, g.cap, A.chunk, acc, g.overflow, swork,
                                   g.perm, g.begin_p, vis);
            });
    }
    if (vis) hipLaunchKernelGGL(k_vis_resolve, dim3(2048), dim3(256), 0, st, sq, vis, g.begin_p, g.end_p, g.cap, acc);
}

// One plain frame.  Per pass: ray generation, then for each depth the
// closest-hit traversal and the shading, which appends the depth's shadow rays
// to one deferred queue (shadow rays feed only the accumulator, so nothing
// waits for them); after the last bounce the queue is binned by light and
// origin cell and traced in one launch, free of the per-depth launch tails.
static rt_status enqueue_frame(const FrameArgs& A, hipStream_t st) {
    const Plan& pl = A.pl;
    uint32_t* ctr = reinterpret_cast<uint32_t*>(A.ws + pl.off_ctr);
    float* acc = reinterpret_cast<float*>(A.ws + pl.off_acc);
    RayQ q[2] = {ray_queue(A.ws + pl.off_q[0], pl.qcap), ray_queue(A.ws + pl.off_q[1], pl.qcap)};
    HitQ hq = hit_queue(A.ws + pl.off_hit, pl.qcap);
    ShadowQ sq = shadow_queue(A.ws + pl.off_s, pl.scap);
    int32_t* overflow = reinterpret_cast<int32_t*>(A.ws + pl.off_stack);
    const int gx = A.gx, shade_blocks = A.shade_blocks;
    unsigned long long* work = A.stats ? reinterpret_cast<unsigned long long*>(&A.stats->node_visits) : nullptr;
    unsigned long long* swork = A.stats ? reinterpret_cast<unsigned long long*>(&A.stats->shadow_node_visits) : nullptr;
    const size_t stride = a256(4 * (size_t)pl.scap);
    uint32_t* bins = reinterpret_cast<uint32_t*>(A.ws + pl.off_bins);
    const int nb = std::max(1, std::min(A.sc.n_lights, 32)) * A.shc.bin_c * A.shc.bin_c * A.shc.bin_c;
    if (A.bin_shadows) sq.key = reinterpret_cast<uint32_t*>(A.ws + pl.off_s2);
    ShadowSegment seg;
    seg.begin_p = nullptr;
    seg.cap = pl.scap;
    seg.end_p = ctr + kCtrShadowAll;
    seg.cursor = xcd_cursor(ctr, kCtrShadowAllCur);
    seg.perm = A.bin_shadows ? reinterpret_cast<uint32_t*>(A.ws + pl.off_s2 + stride) : nullptr;
    seg.bins = bins;
    seg.overflow = reinterpret_cast<int32_t*>(A.ws + pl.off_stack + pl.stack_bytes);
    seg.grid = A.gs;
    const int64_t n3 = 3 * pl.nacc;
    hipLaunchKernelGGL(k_clear_acc, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, acc, n3, ctr + kCtrAccum);
    if (A.shc.light_pts) {
        const int n = A.spp * A.sc.n_lights;
        hipLaunchKernelGGL(k_light_points, dim3((n + 255) / 256), dim3(256), 0, st, A.sc.lights, A.sc.n_lights,
                           A.spp, A.shc.seed, ctr + kCtrFrame, const_cast<float4*>(A.shc.light_pts));
    }
    const int tiles_x = (int)tiles_x_of(A.cam.W, A.tile), tiles_y = (int)tiles_y_of(A.cam.H, A.tile);
    for (int pass = 0; pass < pl.passes; ++pass) {
        const int s0 = pass * pl.spp_pass;
        const int ns = std::min(pl.spp_pass, A.spp - s0);
        clear_counters(ctr, st);
        const uint32_t nthreads = (uint32_t)((int64_t)tiles_x * tiles_y * ns * 64);
        launch_raygen(A, s0, ns, tiles_x, nthreads, q[0], ctr, pl.qcap, acc, st);
        for (int k = 0; k <= A.shc.max_depth; ++k) {
            RayQ& qi = q[k & 1];
            RayQ& qo = q[(k + 1) & 1];
            {
                KernelTimer kt(A.time_kernels, st, 0);
                if (A.count_work)
                    hipLaunchKernelGGL((k_extend<true, false>), dim3(gx), dim3(256), A.lds, st, A.sc, nullptr, qi, hq,
                                       ctr + kCtrRays + k, xcd_cursor(ctr, kCtrRayCur + k), pl.qcap, A.chunk,
                                       overflow, work);
                else if (k > 0)
                    by_layout(A.sc.wide, [&](auto L) {
                        hipLaunchKernelGGL(k_extend_deep<decltype(L)::value>, dim3(A.gxd), dim3(256), 0, st, A.sc, qi,
                                           hq, ctr + kCtrRays + k, xcd_cursor(ctr, kCtrRayCur + k), pl.qcap, A.chunk,
                                           overflow);
                    });
                else
                    by_layout(A.sc.wide, [&](auto L) {
                        hipLaunchKernelGGL((k_extend<false, false, decltype(L)::value>), dim3(gx), dim3(256), A.lds,
                                           st, A.sc, nullptr, qi, hq, ctr + kCtrRays + k,
                                           xcd_cursor(ctr, kCtrRayCur + k), pl.qcap, A.chunk, overflow, work);
                    });
            }
            {
                KernelTimer kt(A.time_kernels, st, 1);
                if (A.shc.gi)
                    hipLaunchKernelGGL((k_shade<false, true>), dim3(shade_blocks), dim3(256), 0, st, A.sc, A.shc,
                                       nullptr, qi, hq, ctr, k, qo, sq, acc);
                else
                    hipLaunchKernelGGL((k_shade<false, false>), dim3(shade_blocks), dim3(256), 0, st, A.sc, A.shc,
                                       nullptr, qi, hq, ctr, k, qo, sq, acc);
            }
        }
        enqueue_shadow_segment(A, sq, seg, nb, acc, swork, st);
        hipLaunchKernelGGL(k_stats, dim3(1), dim3(64), 0, st, ctr, A.stats, A.shc.max_depth, 0);
    }
    hipLaunchKernelGGL(k_resolve, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, acc, A.out_rgb, n3,
                       A.shc.per_sample ? 1.0f : 1.0f / (float)A.spp, ctr + kCtrAccum);
    HIP_TRY(hipGetLastError());
    return RT_OK;
}

// Captured frames, keyed by everything the launch sequence depends on.
struct GraphKey {
    std::vector<uint8_t> bytes;
    bool operator<(const GraphKey& o) const { return bytes < o.bytes; }
};
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
};

static std::mutex g_graph_mu;
static std::map<GraphKey, GraphEntry> g_graphs;

template <class T>
static void put(std::vector<uint8_t>& v, const T& x) {
    const uint8_t* p = reinterpret_cast<const uint8_t*>(&x);
    v.insert(v.end(), p, p + sizeof(T));
}

static rt_status launch_frame(const FrameArgs& A, hipStream_t st, bool use_graph, uint64_t uid) {
    if (!use_graph) return enqueue_frame(A, st);
    GraphKey key;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    put(key.bytes, dev);
    put(key.bytes, uid);
    put(key.bytes, A.sc);
    put(key.bytes, A.cam);
    put(key.bytes, A.shc);
    put(key.bytes, A.pl);
    put(key.bytes, A.ws);
    put(key.bytes, A.stats);
    put(key.bytes, A.out_rgb);
    put(key.bytes, A.out_ids);
    put(key.bytes, A.count_work);
    put(key.bytes, A.spp);
    put(key.bytes, A.gx);
    put(key.bytes, A.gxd);
    put(key.bytes, A.gs);
    put(key.bytes, A.shade_blocks);
    put(key.bytes, A.chunk);
    put(key.bytes, A.bin_shadows);
    std::lock_guard<std::mutex> g(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        GraphEntry e;
        HIP_TRY(hipStreamCreateWithFlags(&e.cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(e.cap_stream, hipStreamCaptureModeThreadLocal));
        rt_status rs = enqueue_frame(A, e.cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t ee = hipStreamEndCapture(e.cap_stream, &graph);
        if (rs != RT_OK) return rs;
        if (ee != hipSuccess) {
            set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
            return RT_ERR_HIP;
        }
        HIP_TRY(hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0));
        HIP_TRY(hipGraphDestroy(graph));
        if (g_graphs.size() > 64) {   // bound the cache
            for (auto& kv : g_graphs) {
                (void)hipGraphExecDestroy(kv.second.exec);
                (void)hipStreamDestroy(kv.second.cap_stream);
            }
            g_graphs.clear();
        }
        it = g_graphs.emplace(key, e).first;
    }
    HIP_TRY(hipGraphLaunch(it->second.exec, st));
    return RT_OK;
}

// ---------------------------------------------------------------------------
// batched frames: many scenes in one wavefront
// ---------------------------------------------------------------------------
struct BatchPlan {
    int n = 0;
    uint32_t n_rays = 0;        // primary slots of all scenes (every sample in one pass)
    uint64_t n_acc = 0;
    uint32_t qcap = 0, scap = 0;
    int dmax = 0, stack_max = 0;
    bool any_gi = false;        // some scene renders with global illumination
    size_t off_tab = 0, off_ctr = 0, off_acc = 0, off_q[2] = {0, 0}, off_hit = 0, off_s = 0, off_stack = 0, total = 0;
    size_t off_lpts = 0;
    uint32_t n_lpts = 0;        // light-point entries of the scenes with area lights
};

static bool make_batch_plan(const rt_scene* const* scenes, const rt_camera* cams, const rt_params* params, int32_t n,
                            float* const* out_rgb, int32_t* const* out_ids, BatchPlan& bp,
                            std::vector<BatchScene>* table, std::string& why) {
    std::memset(&bp, 0, sizeof bp);
    if (!scenes || !cams || !params || n <= 0 || n > 4096) {
        why = "need 1..4096 scenes and non-NULL scenes, cams, params";
        return false;
    }
    const rt_params& p0 = params[0];
    const bool per_sample = (p0.flags & RT_FLAG_PER_SAMPLE) != 0;
    uint64_t rays = 0, acc = 0, lpts = 0;
    int max_lights = 1;
    if (table) table->resize(n);
    for (int i = 0; i < n; ++i) {
        const rt_scene* sc = scenes[i];
        const rt_camera& cam = cams[i];
        const rt_params& p = params[i];
        if (!sc) {
            why = "scene " + std::to_string(i) + " is NULL";
            return false;
        }
        if (cam.width <= 0 || cam.height <= 0 || p.spp < 1 || p.spp > 65535 || p.max_depth < 0 ||
            p.max_depth > RT_STATS_MAX_DEPTH - 2 || !(cam.vfov_deg > 0.0f && cam.vfov_deg < 180.0f) ||
            !std::isfinite(p.eps) || p.eps < 0.0f || !tile_ok(p.tile)) {
            why = "invalid camera or parameters of scene " + std::to_string(i);
            return false;
        }
        const SceneHost& h = sc->h;
        const int64_t tiles_x = tiles_x_of(cam.width, p.tile), tiles_y = tiles_y_of(cam.height, p.tile);
        const uint64_t nr = (uint64_t)tiles_x * tiles_y * 64 * p.spp;
        const uint64_t npix = (uint64_t)cam.width * cam.height;
        const uint64_t na = per_sample ? npix * p.spp : npix;
        if (table) {
            if (!h.dev) {
                why = "scene " + std::to_string(i) + " is not uploaded";
                return false;
            }
            if (!out_rgb[i]) {
                why = "out_rgb[" + std::to_string(i) + "] is NULL";
                return false;
            }
            BatchScene& B = (*table)[i];
            std::memset(&B, 0, sizeof B);
            B.sc = h.dev_view();
            for (int c = 0; c < 3; ++c) B.shc.bg[c] = p.bg[c];
            B.shc.eps = p.eps;
            B.shc.seed = p.seed;
            B.shc.max_depth = p.max_depth;
            B.shc.spp = p.spp;
            B.shc.per_sample = per_sample ? 1 : 0;
            B.shc.acc_off = (uint32_t)acc;
            B.shc.out_ids = out_ids ? out_ids[i] : nullptr;
            B.shc.defer_shadow = 1;   // one shadow queue for every scene and depth, traced after the bounces
            B.shc.gi = (p.flags & RT_FLAG_GI) ? 1 : 0;
            camera_consts(cam, p, B.cam);
            B.ray_off = (uint32_t)rays;
            B.n_rays = (uint32_t)nr;
            B.n_acc = (uint32_t)na;
            B.tiles_x = (int)tiles_x;
            B.inv_spp = per_sample ? 1.0f : 1.0f / (float)p.spp;
            B.out_rgb = out_rgb[i];
            B.shc.seed = p.seed;
            B.lpt_first = (uint32_t)lpts;
            B.lpt_count = h.area_lights ? (uint32_t)(p.spp * h.n_lights) : 0u;
        }
        if (h.area_lights) lpts += (uint64_t)p.spp * h.n_lights;
        rays += nr;
        acc += na;
        bp.dmax = std::max(bp.dmax, p.max_depth);
        bp.any_gi = bp.any_gi || (p.flags & RT_FLAG_GI);
        bp.stack_max = std::max(bp.stack_max, h.stack_size);
        max_lights = std::max(max_lights, h.n_lights);
    }
    const double qf = p0.queue_factor > 0.0f ? std::max(1.0f, p0.queue_factor) : 2.0;
    const double qcap = std::ceil((double)rays * qf);
    // scenes in path tracing need room for a shadow ray per light at every depth of every path
    const double scap = std::max(qcap * max_lights, bp.any_gi ? (double)rays * (bp.dmax + 1) * max_lights : 0.0);
    if (rays >= (1ull << 32) || acc >= (1ull << 32) || qcap > 4.0e9 || scap > 4.0e9) {
        why = "batch too large for one wavefront (more than 2^32 rays or queue entries)";
        return false;
    }
    bp.n = n;
    bp.n_rays = (uint32_t)rays;
    bp.n_acc = acc;
    bp.qcap = (uint32_t)qcap;
    bp.scap = (uint32_t)scap;
    size_t off = 0;
    bp.off_tab = off;
    off = a256(off + sizeof(BatchScene) * n);
    bp.off_ctr = off;
    off = a256(off + 4 * kCtrTotal);
    bp.off_acc = off;
    off = a256(off + 12 * (size_t)acc);
    for (int b = 0; b < 2; ++b) {
        bp.off_q[b] = off;
        off = a256(off + ray_queue_bytes(bp.qcap));
    }
    bp.off_hit = off;
    off = a256(off + 2 * a256(4 * (size_t)bp.qcap));
    bp.off_s = off;
    off = a256(off + shadow_queue_bytes(bp.scap));
    bp.off_stack = off;
    off = a256(off + 4 * (size_t)kMaxPersistentThreads * std::max(0, bp.stack_max - kSplitLds));
    bp.off_lpts = off;
    bp.n_lpts = (uint32_t)std::min<uint64_t>(lpts, 0xFFFFFFFFu);
    off = a256(off + 16 * (size_t)lpts);
    bp.total = off;
    if (table && p0.workspace)
        for (BatchScene& B : *table)
            B.shc.light_pts = B.lpt_count ? reinterpret_cast<const float4*>(
                                                static_cast<uint8_t*>(p0.workspace) + bp.off_lpts) + B.lpt_first
                                          : nullptr;
    return true;
}

struct BatchArgs {
    BatchPlan pl;
    uint8_t* ws;
    rt_stats* stats;
    bool count_work, time_kernels, time_shadow = false;
    uint32_t chunk;
    int gx, gs, shade_blocks;
};

static rt_status batch_grids(BatchArgs& B) {
    rt_status s1 = B.count_work ? persistent_grid(k_extend<true, true>, 0, B.gx)
                                : persistent_grid(k_extend<false, true>, 0, B.gx);
    if (s1 != RT_OK) return s1;
    s1 = B.count_work ? persistent_grid(k_shadow<true, true>, 0, B.gs) : persistent_grid(k_shadow<false, true>, 0, B.gs);
    if (s1 != RT_OK) return s1;
    B.gx = std::min<int>(B.gx, (int)(kMaxPersistentThreads / 256));
    B.gs = std::min<int>(B.gs, (int)(kMaxPersistentThreads / 256));
    B.gx = (int)std::min<int64_t>(B.gx, std::max<int64_t>(kXcd, ((int64_t)B.pl.qcap + 255) / 256));
    B.gs = (int)std::min<int64_t>(B.gs, std::max<int64_t>(kXcd, ((int64_t)B.pl.scap + 255) / 256));
    DevInfo di;
    s1 = device_info(di);
    if (s1 != RT_OK) return s1;
    B.shade_blocks = (int)std::max<int64_t>(1, std::min<int64_t>((B.pl.qcap + 255) / 256, (int64_t)di.cus * 16));
    return RT_OK;
}

// The scene table goes through a pinned staging buffer; the previous upload
// must have completed before the buffer is rewritten.
static std::mutex g_stage_mu;
static void* g_stage = nullptr;
static size_t g_stage_bytes = 0;
static hipEvent_t g_stage_done = nullptr;

static rt_status upload_table(const std::vector<BatchScene>& table, uint8_t* dst, hipStream_t st) {
    std::lock_guard<std::mutex> g(g_stage_mu);
    const size_t bytes = sizeof(BatchScene) * table.size();
    if (g_stage_done) HIP_TRY(hipEventSynchronize(g_stage_done));
    else HIP_TRY(hipEventCreateWithFlags(&g_stage_done, hipEventDisableTiming));
    if (g_stage_bytes < bytes) {
        if (g_stage) HIP_TRY(hipHostFree(g_stage));
        g_stage = nullptr;
        g_stage_bytes = 0;
        HIP_TRY(hipHostMalloc(&g_stage, bytes, hipHostMallocDefault));
        g_stage_bytes = bytes;
    }
    std::memcpy(g_stage, table.data(), bytes);
    HIP_TRY(hipMemcpyAsync(dst, g_stage, bytes, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(g_stage_done, st));
    return RT_OK;
}

static rt_status enqueue_batch(const BatchArgs& B, hipStream_t st) {
    const BatchPlan& pl = B.pl;
    const BatchScene* tab = reinterpret_cast<const BatchScene*>(B.ws + pl.off_tab);
    uint32_t* ctr = reinterpret_cast<uint32_t*>(B.ws + pl.off_ctr);
    float* acc = reinterpret_cast<float*>(B.ws + pl.off_acc);
    RayQ q[2] = {ray_queue(B.ws + pl.off_q[0], pl.qcap), ray_queue(B.ws + pl.off_q[1], pl.qcap)};
    HitQ hq = hit_queue(B.ws + pl.off_hit, pl.qcap);
    ShadowQ sq = shadow_queue(B.ws + pl.off_s, pl.scap);
    int32_t* overflow = reinterpret_cast<int32_t*>(B.ws + pl.off_stack);
    unsigned long long* work = B.stats ? reinterpret_cast<unsigned long long*>(&B.stats->node_visits) : nullptr;
    unsigned long long* swork = B.stats ? reinterpret_cast<unsigned long long*>(&B.stats->shadow_node_visits) : nullptr;
    DevScene none;
    std::memset(&none, 0, sizeof none);
    ShadeConst c0;
    std::memset(&c0, 0, sizeof c0);
    c0.qcap = pl.qcap;
    c0.scap = pl.scap;
    const uint64_t n3 = 3 * pl.n_acc;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, acc, (int64_t)n3, 0.0f);
    clear_counters(ctr, st);
    if (pl.n_lpts)
        hipLaunchKernelGGL(k_light_points_batch, dim3((pl.n_lpts + 255) / 256), dim3(256), 0, st, tab, pl.n, pl.n_lpts);
    hipLaunchKernelGGL(k_raygen_batch, dim3((pl.n_rays + 255) / 256), dim3(256), 0, st, tab, pl.n, pl.n_rays, q[0], ctr,
                       pl.qcap);
    for (int k = 0; k <= pl.dmax; ++k) {
        RayQ& qi = q[k & 1];
        RayQ& qo = q[(k + 1) & 1];
        {
            KernelTimer kt(B.time_kernels, st, 0);
            if (B.count_work)
                hipLaunchKernelGGL((k_extend<true, true>), dim3(B.gx), dim3(256), 0, st, none, tab, qi, hq,
                                   ctr + kCtrRays + k, xcd_cursor(ctr, kCtrRayCur + k), pl.qcap, B.chunk, overflow,
                                   work);
            else
                hipLaunchKernelGGL((k_extend<false, true>), dim3(B.gx), dim3(256), 0, st, none, tab, qi, hq,
                                   ctr + kCtrRays + k, xcd_cursor(ctr, kCtrRayCur + k), pl.qcap, B.chunk, overflow,
                                   work);
        }
        {
            KernelTimer kt(B.time_kernels, st, 1);
            if (B.pl.any_gi)
                hipLaunchKernelGGL((k_shade<true, true>), dim3(B.shade_blocks), dim3(256), 0, st, none, c0, tab, qi, hq,
                                   ctr, k, qo, sq, acc);
            else
                hipLaunchKernelGGL((k_shade<true, false>), dim3(B.shade_blocks), dim3(256), 0, st, none, c0, tab, qi,
                                   hq, ctr, k, qo, sq, acc);
        }
    }
    {   // the deferred shadow rays of every scene and depth
        KernelTimer kt(B.time_kernels || B.time_shadow, st, 2);
        if (B.count_work)
            hipLaunchKernelGGL((k_shadow<true, true>), dim3(B.gs), dim3(256), 0, st, none, tab, sq,
                               ctr + kCtrShadowAll, xcd_cursor(ctr, kCtrShadowAllCur), pl.scap, B.chunk, acc,
                               overflow, swork);
        else
            hipLaunchKernelGGL((k_shadow<false, true>), dim3(B.gs), dim3(256), 0, st, none, tab, sq,
                               ctr + kCtrShadowAll, xcd_cursor(ctr, kCtrShadowAllCur), pl.scap, B.chunk, acc,
                               overflow, swork);
    }
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(64), 0, st, ctr, B.stats, pl.dmax, 0);
    hipLaunchKernelGGL(k_resolve_batch, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, tab, pl.n, acc, n3);
    HIP_TRY(hipGetLastError());
    return RT_OK;
}

static rt_status launch_batch(const BatchArgs& B, hipStream_t st, bool use_graph) {
    if (!use_graph) return enqueue_batch(B, st);
    GraphKey key;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const uint32_t tag = 0xBA7C4u;
    put(key.bytes, tag);
    put(key.bytes, dev);
    put(key.bytes, B.pl);
    put(key.bytes, B.ws);
    put(key.bytes, B.stats);
    put(key.bytes, B.count_work);
    put(key.bytes, B.chunk);
    put(key.bytes, B.gx);
    put(key.bytes, B.gs);
    put(key.bytes, B.shade_blocks);
    std::lock_guard<std::mutex> g(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        GraphEntry e;
        HIP_TRY(hipStreamCreateWithFlags(&e.cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(e.cap_stream, hipStreamCaptureModeThreadLocal));
        rt_status rs = enqueue_batch(B, e.cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t ee = hipStreamEndCapture(e.cap_stream, &graph);
        if (rs != RT_OK) return rs;
        if (ee != hipSuccess) {
            set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
            return RT_ERR_HIP;
        }
        HIP_TRY(hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0));
        HIP_TRY(hipGraphDestroy(graph));
        it = g_graphs.emplace(key, e).first;
    }
    HIP_TRY(hipGraphLaunch(it->second.exec, st));
    return RT_OK;
}

// ---------------------------------------------------------------------------
// learned form: host side
// ---------------------------------------------------------------------------
rt_status mlp_infer_launch(const uint16_t* w, const uint16_t* x, int64_t cap, const uint32_t* count, const uint32_t* pix,
                           const float* wt, float* acc, hipStream_t st);
rt_status mlp_grad_launch(const uint16_t* w, const uint16_t* x, const float* target, int64_t n, int64_t n_total,
                          const uint32_t* count, int64_t count_base, float* dw, float* loss, hipStream_t st);
rt_status mlp_adam_dev_launch(float* w, uint16_t* wb, float* m, float* v, float* g, const uint32_t* step_p, float lr,
                              float b1, float b2, float eps, hipStream_t st);
rt_status mlp_health_launch(const float* w, const float* m, const float* v, const uint32_t* loss_bits, int steps,
                            uint32_t* health, hipStream_t st);

constexpr int kMlpParams = 5 * 64 * 64 + 3 * 64;
constexpr int kTargetGrowth = 4;    // target-wavefront queue capacity per training sample

static bool cache_layout(int32_t cap, rt_cache_layout& L) {
    if (cap <= 0 || cap > (1 << 24)) return false;
    std::memset(&L, 0, sizeof L);
    size_t off = 0;
    L.w_master = off;
    off = a256(off + 4 * (size_t)kMlpParams);
    L.w_bf16 = off;
    off = a256(off + 2 * (size_t)kMlpParams);
    L.m = off;
    off = a256(off + 4 * (size_t)kMlpParams);
    L.v = off;
    off = a256(off + 4 * (size_t)kMlpParams);
    L.grad = off;
    off = a256(off + 4 * (size_t)kMlpParams);
    L.counters = off;
    off = a256(off + 4 * 64);
    L.train_rays = off;
    off = a256(off + 24 * (size_t)cap);
    L.train_feats = off;
    off = a256(off + 128 * (size_t)cap);
    L.train_targets = off;
    off = a256(off + 12 * (size_t)cap);
    L.train_pix = off;
    off = a256(off + 4 * (size_t)cap);
    L.total = off;
    L.capacity = cap;
    return true;
}

struct CachePlan {
    Plan base;
    rt_cache c;            // defaults filled in
    rt_cache_layout L;
    uint32_t rec_cap = 0, tcap = 0, tscap = 0;
    size_t off_rec = 0, off_tq[2] = {0, 0}, off_thit = 0, off_ts = 0, off_tbin = 0, off_tbins = 0, off_tctr = 0,
           off_fbctr = 0, total = 0;
};

static bool make_cache_plan(const SceneHost& h, const rt_camera& cam, const rt_params& p, const rt_cache* cache,
                            CachePlan& cp, std::string& why) {
    std::memset(&cp, 0, sizeof cp);
    if (!cache || !cache->state) {
        why = "cache and cache->state are required";
        return false;
    }
    rt_cache c = *cache;
    if (c.mode != RT_CACHE_INFER && c.mode != RT_CACHE_TRAIN) {
        why = "cache mode must be RT_CACHE_INFER or RT_CACHE_TRAIN";
        return false;
    }
    if (c.depth <= 0) c.depth = 2;
    if (c.full_depth <= 0) c.full_depth = 8;
    if (c.train_samples <= 0) c.train_samples = 65536;
    if (c.train_steps <= 0) c.train_steps = 4;
    if (!(c.lr > 0.0f)) c.lr = 1e-3f;
    if (!(c.b1 > 0.0f)) c.b1 = 0.9f;
    if (!(c.b2 > 0.0f)) c.b2 = 0.999f;
    if (!(c.eps > 0.0f)) c.eps = 1e-8f;
    if (c.depth > RT_STATS_MAX_DEPTH - 2 || c.full_depth > RT_STATS_MAX_DEPTH - 2 || c.full_depth < c.depth ||
        c.train_steps > 16) {
        why = "cache depth / full_depth must be in [1, 14] with full_depth >= depth; train_steps <= 16";
        return false;
    }
    bool zero = true;
    for (int k = 0; k < 3; ++k) zero = zero && c.bounds_lo[k] == 0.0f && c.bounds_hi[k] == 0.0f;
    if (zero)
        for (int k = 0; k < 3; ++k) {
            c.bounds_lo[k] = h.info.bounds_lo[k];
            c.bounds_hi[k] = h.info.bounds_hi[k];
        }
    for (int k = 0; k < 3; ++k)
        if (!(c.bounds_hi[k] > c.bounds_lo[k])) c.bounds_hi[k] = c.bounds_lo[k] + 1.0f;
    rt_params q = p;
    q.samples_per_pass = p.spp;   // cache frames trace every sample in one pass
    // path tracing: the image's paths are shaded above the cache depth, and by the fallback chain (an
    // unhealthy cache) from it to max_depth; the larger of the two bounds the deferred shadow queue
    if (p.flags & RT_FLAG_GI)
        q.max_depth = std::max(0, std::min(p.max_depth, std::max(c.depth - 1, p.max_depth - c.depth)));
    if (!make_plan(h, cam, q, cp.base, why)) return false;
    cp.c = c;
    if (!cache_layout(c.train_samples, cp.L)) {
        why = "train_samples must be in [1, 2^24]";
        return false;
    }
    const Plan& pl = cp.base;
    cp.rec_cap = pl.qcap;
    cp.tcap = (uint32_t)std::min<uint64_t>(4000000000ull, (uint64_t)c.train_samples * kTargetGrowth);
    cp.tscap = (uint32_t)std::min<uint64_t>(4000000000ull, (uint64_t)cp.tcap * std::max(1, h.n_lights));
    if (p.flags & RT_FLAG_GI) {   // target paths: one ray per depth, a shadow ray per light at each of their hits
        cp.tcap = (uint32_t)c.train_samples;
        cp.tscap = (uint32_t)std::min<uint64_t>(
            4000000000ull, (uint64_t)c.train_samples * (c.full_depth - c.depth + 1) * std::max(1, h.n_lights));
    }
    size_t off = pl.total;
    cp.off_rec = off;
    off = a256(off + (size_t)cp.rec_cap * (128 + 4 + 12 + 4) + 4 * 256);
    for (int b = 0; b < 2; ++b) {
        cp.off_tq[b] = off;
        off = a256(off + ray_queue_bytes(cp.tcap));
    }
    cp.off_thit = off;
    off = a256(off + 2 * a256(4 * (size_t)cp.tcap));
    cp.off_ts = off;
    off = a256(off + shadow_queue_bytes(cp.tscap));
    cp.off_tbin = off;    // keys and order of the targets' deferred shadow queue
    off = a256(off + 2 * a256(4 * (size_t)cp.tscap));
    cp.off_tbins = off;   // its per-bin counts and first slots
    off = a256(off + 2 * 4 * (size_t)kBinMax);
    cp.off_tctr = off;
    off = a256(off + 4 * kCtrTotal);
    cp.off_fbctr = off;   // counters of the fallback chain
    off = a256(off + 4 * kCtrTotal);
    cp.total = off;
    return true;
}

static CacheRec cache_records(uint8_t* base, uint32_t cap) {
    CacheRec r;
    r.feats = reinterpret_cast<uint16_t*>(base);
    size_t off = a256((size_t)cap * 128);
    r.pix = reinterpret_cast<uint32_t*>(base + off);
    off = a256(off + 4 * (size_t)cap);
    r.w = reinterpret_cast<float*>(base + off);
    off = a256(off + 12 * (size_t)cap);
    r.src = reinterpret_cast<uint32_t*>(base + off);
    r.cap = cap;
    return r;
}

struct CacheArgs {
    FrameArgs F;
    CachePlan cp;
    uint8_t* state;
};

static rt_status enqueue_cached(const CacheArgs& C, hipStream_t st) {
    const FrameArgs& A = C.F;
    const Plan& pl = A.pl;
    const CachePlan& cp = C.cp;
    const rt_cache& cc = cp.c;
    uint32_t* ctr = reinterpret_cast<uint32_t*>(A.ws + pl.off_ctr);
    float* acc = reinterpret_cast<float*>(A.ws + pl.off_acc);
    RayQ q[2] = {ray_queue(A.ws + pl.off_q[0], pl.qcap), ray_queue(A.ws + pl.off_q[1], pl.qcap)};
    HitQ hq = hit_queue(A.ws + pl.off_hit, pl.qcap);
    ShadowQ sq = shadow_queue(A.ws + pl.off_s, pl.scap);
    int32_t* overflow = reinterpret_cast<int32_t*>(A.ws + pl.off_stack);
    const CacheRec rec = cache_records(A.ws + cp.off_rec, cp.rec_cap);
    uint8_t* S = C.state;
    const rt_cache_layout& L = cp.L;
    const uint16_t* w_bf16 = reinterpret_cast<const uint16_t*>(S + L.w_bf16);
    uint32_t* counters = reinterpret_cast<uint32_t*>(S + L.counters);
    unsigned long long* work = A.stats ? reinterpret_cast<unsigned long long*>(&A.stats->node_visits) : nullptr;
    unsigned long long* swork = A.stats ? reinterpret_cast<unsigned long long*>(&A.stats->shadow_node_visits) : nullptr;
    const int cd = cc.depth;

    // one bounce of a wavefront: closest hits and shading; the shading appends
    // its shadow rays to the chain's deferred queue (counters c_)
    auto bounce = [&](RayQ& qi, RayQ& qo, HitQ& h, ShadowQ& sh, uint32_t* c_, const ShadeConst& shc, float* acc_,
                      int k) {
        {
            KernelTimer kt(A.time_kernels, st, 0);
            if (A.count_work)
                hipLaunchKernelGGL((k_extend<true, false>), dim3(A.gx), dim3(256), 0, st, A.sc, nullptr, qi, h,
                                   c_ + kCtrRays + k, xcd_cursor(c_, kCtrRayCur + k), shc.qcap, A.chunk, overflow,
                                   work);
            else
                by_layout(A.sc.wide, [&](auto L) {
                    hipLaunchKernelGGL((k_extend<false, false, decltype(L)::value>), dim3(A.gx), dim3(256), 0, st,
                                       A.sc, nullptr, qi, h, c_ + kCtrRays + k, xcd_cursor(c_, kCtrRayCur + k),
                                       shc.qcap, A.chunk, overflow, work);
                });
        }
        {
            KernelTimer kt(A.time_kernels, st, 1);
            if (shc.gi)
                hipLaunchKernelGGL((k_shade<false, true>), dim3(A.shade_blocks), dim3(256), 0, st, A.sc, shc, nullptr,
                                   qi, h, c_, k, qo, sh, acc_);
            else
                hipLaunchKernelGGL((k_shade<false, false>), dim3(A.shade_blocks), dim3(256), 0, st, A.sc, shc, nullptr,
                                   qi, h, c_, k, qo, sh, acc_);
        }
    };
    // the deferred shadow queue of a chain, binned and traced once
    const int nb = std::max(1, std::min(A.sc.n_lights, 32)) * A.shc.bin_c * A.shc.bin_c * A.shc.bin_c;
    auto shadows = [&](const ShadowQ& sh, uint32_t* c_, uint32_t cap, uint32_t* perm, uint32_t* bins, float* acc_) {
        ShadowSegment g;
        g.begin_p = nullptr;
        g.end_p = c_ + kCtrShadowAll;
        g.cap = cap;
        g.cursor = xcd_cursor(c_, kCtrShadowAllCur);
        g.perm = perm;
        g.bins = bins;
        g.overflow = overflow;
        g.grid = A.gs;
        enqueue_shadow_segment(A, sh, g, nb, acc_, swork, st);
    };
    const size_t sstride = a256(4 * (size_t)pl.scap);
    sq.key = reinterpret_cast<uint32_t*>(A.ws + pl.off_s2);

    const int64_t n3 = 3 * pl.nacc;
    uint32_t* ctr_fb = reinterpret_cast<uint32_t*>(A.ws + cp.off_fbctr);
    uint32_t* health = counters + kCacheHealth;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, acc, n3, 0.0f);
    clear_counters(ctr, st);
    clear_counters(ctr_fb, st);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, ctr + kCtrRec, 1);
    if (A.shc.light_pts) {
        const int n = A.spp * A.sc.n_lights;
        hipLaunchKernelGGL(k_light_points, dim3((n + 255) / 256), dim3(256), 0, st, A.sc.lights, A.sc.n_lights,
                           A.spp, A.shc.seed, ctr + kCtrFrame, const_cast<float4*>(A.shc.light_pts));
    }
    const int tiles_x = (int)tiles_x_of(A.cam.W, A.tile), tiles_y = (int)tiles_y_of(A.cam.H, A.tile);
    const uint32_t nthreads = (uint32_t)((int64_t)tiles_x * tiles_y * A.spp * 64);
    launch_raygen(A, 0, A.spp, tiles_x, nthreads, q[0], ctr, pl.qcap, acc, st);
    for (int k = 0; k < cd; ++k) bounce(q[k & 1], q[(k + 1) & 1], hq, sq, ctr, A.shc, acc, k);
    shadows(sq, ctr, pl.scap, reinterpret_cast<uint32_t*>(A.ws + pl.off_s2 + sstride),
            reinterpret_cast<uint32_t*>(A.ws + pl.off_bins), acc);
    // depth cd: closest hits, then cache queries instead of shading
    {
        KernelTimer kt(A.time_kernels, st, 0);
        by_layout(A.sc.wide, [&](auto L) {
            hipLaunchKernelGGL((k_extend<false, false, decltype(L)::value>), dim3(A.gx), dim3(256), 0, st, A.sc,
                               nullptr, q[cd & 1], hq, ctr + kCtrRays + cd, xcd_cursor(ctr, kCtrRayCur + cd),
                               pl.qcap, A.chunk, overflow, nullptr);
        });
    }
    hipLaunchKernelGGL(k_cache_gate, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, w_bf16, kMlpParams, health, ctr,
                       ctr_fb, cd, A.stats);
    const float ie[3] = {1.0f / (cc.bounds_hi[0] - cc.bounds_lo[0]), 1.0f / (cc.bounds_hi[1] - cc.bounds_lo[1]),
                         1.0f / (cc.bounds_hi[2] - cc.bounds_lo[2])};
    hipLaunchKernelGGL(k_cache_shade, dim3(A.shade_blocks), dim3(256), 0, st, A.sc, A.shc, q[cd & 1], hq, ctr, cd, rec,
                       cc.bounds_lo[0], cc.bounds_lo[1], cc.bounds_lo[2], ie[0], ie[1], ie[2], acc);
    {
        KernelTimer kt(A.time_kernels, st, 3);
        rt_status rs = mlp_infer_launch(w_bf16, rec.feats, rec.cap, ctr + kCtrRec, rec.pix, rec.w, acc, st);
        if (rs != RT_OK) return rs;
    }
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(64), 0, st, ctr, A.stats, cd, 1);
    // Fallback chain: the plain tracer from the cache depth to max_depth.  Its counters hold the depth's hits
    // only when the gate found the cache unhealthy; otherwise every launch finds empty queues and returns.
    // It reuses the image's ray, hit and shadow queues, whose earlier contents are consumed by now.
    {
        KernelTimer kt(A.time_kernels, st, 1);
        if (A.shc.gi)
            hipLaunchKernelGGL((k_shade<false, true>), dim3(A.shade_blocks), dim3(256), 0, st, A.sc, A.shc, nullptr,
                               q[cd & 1], hq, ctr_fb, cd, q[(cd + 1) & 1], sq, acc);
        else
            hipLaunchKernelGGL((k_shade<false, false>), dim3(A.shade_blocks), dim3(256), 0, st, A.sc, A.shc, nullptr,
                               q[cd & 1], hq, ctr_fb, cd, q[(cd + 1) & 1], sq, acc);
    }
    for (int k = cd + 1; k <= A.shc.max_depth; ++k) bounce(q[k & 1], q[(k + 1) & 1], hq, sq, ctr_fb, A.shc, acc, k);
    shadows(sq, ctr_fb, pl.scap, reinterpret_cast<uint32_t*>(A.ws + pl.off_s2 + sstride),
            reinterpret_cast<uint32_t*>(A.ws + pl.off_bins), acc);
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(64), 0, st, ctr_fb, A.stats, A.shc.max_depth, 3);

    if (cc.mode == RT_CACHE_TRAIN) {
        uint32_t* tctr = reinterpret_cast<uint32_t*>(A.ws + cp.off_tctr);
        RayQ tq[2] = {ray_queue(A.ws + cp.off_tq[0], cp.tcap), ray_queue(A.ws + cp.off_tq[1], cp.tcap)};
        HitQ th = hit_queue(A.ws + cp.off_thit, cp.tcap);
        ShadowQ ts = shadow_queue(A.ws + cp.off_ts, cp.tscap);
        ts.key = reinterpret_cast<uint32_t*>(A.ws + cp.off_tbin);
        float* targets = reinterpret_cast<float*>(S + L.train_targets);
        uint16_t* t_feats = reinterpret_cast<uint16_t*>(S + L.train_feats);
        float* t_rays = reinterpret_cast<float*>(S + L.train_rays);
        const uint32_t T = (uint32_t)cc.train_samples;
        clear_counters(tctr, st);
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, counters + 2, 16);
        hipLaunchKernelGGL(k_fill_f32, dim3((3 * T + 255) / 256), dim3(256), 0, st, targets, (int64_t)3 * T, 0.0f);
        hipLaunchKernelGGL(k_cache_select, dim3((T + 255) / 256), dim3(256), 0, st, ctr, rec, q[cd & 1], T, cd,
                           tq[cd & 1], tctr, counters + 1, t_feats, t_rays,
                           reinterpret_cast<uint32_t*>(S + L.train_pix));
        ShadeConst tc = A.shc;
        tc.max_depth = cc.full_depth;
        tc.spp = 1;
        tc.per_sample = 0;
        tc.acc_off = 0;
        tc.out_ids = nullptr;
        tc.qcap = cp.tcap;
        tc.scap = cp.tscap;
        for (int k = cd; k <= cc.full_depth; ++k) bounce(tq[k & 1], tq[(k + 1) & 1], th, ts, tctr, tc, targets, k);
        shadows(ts, tctr, cp.tscap, reinterpret_cast<uint32_t*>(A.ws + cp.off_tbin + a256(4 * (size_t)cp.tscap)),
                reinterpret_cast<uint32_t*>(A.ws + cp.off_tbins), targets);
        hipLaunchKernelGGL(k_stats, dim3(1), dim3(64), 0, st, tctr, A.stats, cc.full_depth, 2);
        const int64_t bs = (T + cc.train_steps - 1) / cc.train_steps;
        float* wm = reinterpret_cast<float*>(S + L.w_master);
        uint16_t* wb = reinterpret_cast<uint16_t*>(S + L.w_bf16);
        float* m = reinterpret_cast<float*>(S + L.m);
        float* v = reinterpret_cast<float*>(S + L.v);
        float* g = reinterpret_cast<float*>(S + L.grad);
        KernelTimer kt(A.time_kernels, st, 4);   // the network's training only (targets are timed as bounces)
        for (int step = 0; step < cc.train_steps; ++step) {
            rt_status rs = mlp_grad_launch(wb, t_feats + (size_t)step * bs * 64, targets + (size_t)step * bs * 3, bs, bs,
                                           counters + 1, step * bs, g, reinterpret_cast<float*>(counters + 2 + step),
                                           st);
            if (rs != RT_OK) return rs;
            rs = mlp_adam_dev_launch(wm, wb, m, v, g, counters + 0, cc.lr, cc.b1, cc.b2, cc.eps, st);
            if (rs != RT_OK) return rs;
        }
        rt_status rs = mlp_health_launch(wm, m, v, counters + 2, cc.train_steps, health, st);
        if (rs != RT_OK) return rs;
    }
    hipLaunchKernelGGL(k_resolve, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, acc, A.out_rgb, n3,
                       A.shc.per_sample ? 1.0f : 1.0f / (float)A.spp, ctr + kCtrAccum);
    HIP_TRY(hipGetLastError());
    return RT_OK;
}

static rt_status launch_cached(const CacheArgs& C, hipStream_t st, bool use_graph, uint64_t uid) {
    if (!use_graph) return enqueue_cached(C, st);
    GraphKey key;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const uint32_t tag = 0xCAC4Eu;
    put(key.bytes, tag);
    put(key.bytes, dev);
    put(key.bytes, uid);
    put(key.bytes, C.F.sc);
    put(key.bytes, C.F.cam);
    put(key.bytes, C.F.shc);
    put(key.bytes, C.F.pl);
    put(key.bytes, C.F.ws);
    put(key.bytes, C.F.stats);
    put(key.bytes, C.F.out_rgb);
    put(key.bytes, C.F.count_work);
    put(key.bytes, C.F.spp);
    put(key.bytes, C.F.gx);
    put(key.bytes, C.F.gs);
    put(key.bytes, C.F.shade_blocks);
    put(key.bytes, C.F.chunk);
    put(key.bytes, C.cp);
    put(key.bytes, C.state);
    std::lock_guard<std::mutex> g(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        GraphEntry e;
        HIP_TRY(hipStreamCreateWithFlags(&e.cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(e.cap_stream, hipStreamCaptureModeThreadLocal));
        rt_status rs = enqueue_cached(C, e.cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t ee = hipStreamEndCapture(e.cap_stream, &graph);
        if (rs != RT_OK) return rs;
        if (ee != hipSuccess) {
            set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
            return RT_ERR_HIP;
        }
        HIP_TRY(hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0));
        HIP_TRY(hipGraphDestroy(graph));
        it = g_graphs.emplace(key, e).first;
    }
    HIP_TRY(hipGraphLaunch(it->second.exec, st));
    return RT_OK;
}

}  // namespace mirt

using namespace mirt;

extern "C" {

size_t rt_render_workspace_bytes(const rt_scene* scene, const rt_camera* cam, const rt_params* params) {
    if (!scene || !cam || !params) {
        set_error("rt_render_workspace_bytes: NULL argument");
        return 0;
    }
    Plan pl;
    std::string why;
    if (!make_plan(scene->h, *cam, *params, pl, why)) {
        set_error("rt_render_workspace_bytes: " + why);
        return 0;
    }
    return pl.total;
}

rt_status rt_render(const rt_scene* scene, const rt_camera* cam, const rt_params* params, float* out_rgb,
                    int32_t* out_hit_ids) {
    if (!scene || !cam || !params || !out_rgb) {
        set_error("rt_render: NULL argument");
        return RT_ERR_INVALID_ARG;
    }
    const SceneHost& h = scene->h;
    if (!h.dev) {
        set_error("rt_render: scene not uploaded (call rt_scene_upload)");
        return RT_ERR_NOT_UPLOADED;
    }
    const rt_params& p = *params;
    if (!std::isfinite(p.eps) || p.eps < 0.0f || !std::isfinite(p.bg[0]) || !std::isfinite(p.bg[1]) ||
        !std::isfinite(p.bg[2])) {
        set_error("rt_render: eps and bg must be finite, eps >= 0");
        return RT_ERR_INVALID_ARG;
    }
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(cam->eye[i]) || !std::isfinite(cam->look_at[i]) || !std::isfinite(cam->up[i])) {
            set_error("rt_render: non-finite camera");
            return RT_ERR_INVALID_ARG;
        }
    if (!(cam->vfov_deg > 0.0f && cam->vfov_deg < 180.0f)) {
        set_error("rt_render: vfov_deg must be in (0, 180)");
        return RT_ERR_INVALID_ARG;
    }
    Plan pl;
    std::memset(&pl, 0, sizeof pl);
    std::string why;
    if (!make_plan(h, *cam, p, pl, why)) {
        set_error("rt_render: " + why);
        return RT_ERR_INVALID_ARG;
    }
    if (!p.workspace || p.workspace_bytes < pl.total) {
        set_error("rt_render: workspace missing or smaller than rt_render_workspace_bytes (" +
                  std::to_string(pl.total) + ")");
        return RT_ERR_CAPACITY;
    }
    if ((reinterpret_cast<uintptr_t>(p.workspace) | reinterpret_cast<uintptr_t>(out_rgb)) & 255) {
        set_error("rt_render: device pointers must be 256-byte aligned");
        return RT_ERR_INVALID_ARG;
    }

    FrameArgs A;
    std::memset(&A, 0, sizeof A);
    A.sc = h.dev_view();
    camera_consts(*cam, p, A.cam);
    A.cam.frame = 0;   // the frame number is read from the workspace, not baked into a captured graph
    for (int i = 0; i < 3; ++i) A.shc.bg[i] = p.bg[i];
    A.shc.eps = p.eps;
    A.shc.seed = p.seed;
    A.shc.max_depth = p.max_depth;
    A.shc.spp = p.spp;
    A.shc.qcap = pl.qcap;
    A.shc.scap = pl.scap;
    A.shc.per_sample = (p.flags & RT_FLAG_PER_SAMPLE) ? 1 : 0;
    A.shc.acc_off = 0;
    A.shc.out_ids = out_hit_ids;
    A.shc.gi = (p.flags & RT_FLAG_GI) ? 1 : 0;
    // depth-0 background / ambient terms summed over the four samples of a pixel in a block
    A.shc.sum_depth0 = (!A.shc.per_sample && pl.spp_pass % 4 == 0) ? 1 : 0;
    defer_and_bin_shadows(A, scene->h);
    A.pl = pl;
    A.ws = static_cast<uint8_t*>(p.workspace);
    A.shc.light_pts = scene->h.area_lights ? reinterpret_cast<const float4*>(A.ws + A.pl.off_lpts) : nullptr;
    A.stats = static_cast<rt_stats*>(p.stats);
    A.out_rgb = out_rgb;
    A.out_ids = out_hit_ids;
    A.count_work = (p.flags & RT_FLAG_COUNT_WORK) != 0;
    A.spp = p.spp;
    A.time_kernels = (p.flags & RT_FLAG_TIME_KERNELS) != 0;
    A.time_shadow = (p.flags & RT_FLAG_TIME_SHADOW) != 0;
    A.chunk = p.queue_chunk > 0 ? (uint32_t)((std::min(p.queue_chunk, 1 << 16) + 63) / 64 * 64) : 128u;
    A.tile = p.tile;
    rt_status rs = frame_grids(A);
    if (rs != RT_OK) return rs;
    hipStream_t st = static_cast<hipStream_t>(p.stream);
    const bool graph = (p.flags & (RT_FLAG_NO_GRAPH | RT_FLAG_TIME_KERNELS | RT_FLAG_TIME_SHADOW)) == 0;
    HIP_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(A.ws + pl.off_ctr + 4 * kCtrFrame), (int)p.frame, 1,
                              st));
    const uint32_t accum = (p.flags & RT_FLAG_ACCUMULATE) ? p.accum_frames : 0u;
    HIP_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(A.ws + pl.off_ctr + 4 * kCtrAccum), (int)accum, 1,
                              st));
    rs = launch_frame(A, st, graph, h.uid);
    if (rs != RT_OK) return rs;
    if (p.flags & RT_FLAG_SYNC) {
        HIP_TRY(hipStreamSynchronize(st));
        if (A.stats) {
            uint32_t status = 0;
            HIP_TRY(hipMemcpy(&status, &A.stats->status, 4, hipMemcpyDeviceToHost));
            if (status) {
                set_error("rt_render: ray queue overflow (status " + std::to_string(status) +
                          "); raise queue_factor");
                return RT_ERR_CAPACITY;
            }
        }
    }
    return RT_OK;
}

static rt_status trace_rays(const rt_scene* scene, const float* rays, int64_t n, float* t, int32_t* id, float* uv,
                            uint8_t* occ, void* workspace, void* stream, bool any) {
    if (!scene || (n > 0 && (!rays || (any ? !occ : (!t || !id)))) || n < 0 || !workspace) {
        set_error("rt_intersect/rt_occluded: invalid argument");
        return RT_ERR_INVALID_ARG;
    }
    if (!scene->h.dev) {
        set_error("rt_intersect/rt_occluded: scene not uploaded");
        return RT_ERR_NOT_UPLOADED;
    }
    if (n == 0) return RT_OK;
    if (n >= ((int64_t)1 << 32) - 64) {
        set_error("rt_intersect/rt_occluded: n must be < 2^32 - 64");
        return RT_ERR_INVALID_ARG;
    }
    const DevScene sc = scene->h.dev_view();
    const size_t lds = (size_t)sc.stack_size * 64 * 4 * 4;
    DevInfo di;
    rt_status rd = device_info(di);
    if (rd != RT_OK) return rd;
    if (lds > (size_t)di.max_lds) {
        set_error("rt_intersect/rt_occluded: the scene's traversal stack does not fit in LDS");
        return RT_ERR_UNSUPPORTED;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint32_t* cursor = static_cast<uint32_t*>(workspace);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, cursor, 1);
    int g = 0;
    rt_status rs = any ? persistent_grid(k_trace_rays<true>, lds, g) : persistent_grid(k_trace_rays<false>, lds, g);
    if (rs != RT_OK) return rs;
    g = (int)std::min<int64_t>(g, (n + 255) / 256);
    float2* uv2 = reinterpret_cast<float2*>(uv);
    if (any)
        hipLaunchKernelGGL(k_trace_rays<true>, dim3(g), dim3(256), lds, st, sc, rays, n, t, id, uv2, occ, cursor);
    else
        hipLaunchKernelGGL(k_trace_rays<false>, dim3(g), dim3(256), lds, st, sc, rays, n, t, id, uv2, occ, cursor);
    HIP_TRY(hipGetLastError());
    return RT_OK;
}

rt_status rt_intersect(const rt_scene* scene, const float* rays, int64_t n, float* t, int32_t* id, float* uv,
                       void* workspace, void* stream) {
    if (uv && (reinterpret_cast<uintptr_t>(uv) & 7u)) {
        set_error("rt_intersect: uv must be 8-byte aligned");
        return RT_ERR_INVALID_ARG;
    }
    return trace_rays(scene, rays, n, t, id, uv, nullptr, workspace, stream, false);
}

rt_status rt_occluded(const rt_scene* scene, const float* rays, int64_t n, uint8_t* occluded, void* workspace,
                      void* stream) {
    return trace_rays(scene, rays, n, nullptr, nullptr, nullptr, occluded, workspace, stream, true);
}


rt_status rt_cache_state_layout(int32_t capacity, rt_cache_layout* out) {
    if (!out || !cache_layout(capacity, *out)) {
        set_error("rt_cache_state_layout: capacity must be in [1, 2^24]");
        return RT_ERR_INVALID_ARG;
    }
    return RT_OK;
}

size_t rt_cache_state_bytes(int32_t capacity) {
    rt_cache_layout L;
    if (!cache_layout(capacity, L)) {
        set_error("rt_cache_state_bytes: capacity must be in [1, 2^24]");
        return 0;
    }
    return L.total;
}

rt_status rt_cache_init(void* state, int32_t capacity, const float* w_host, void* stream) {
    rt_cache_layout L;
    if (!state || !w_host || !cache_layout(capacity, L)) {
        set_error("rt_cache_init: invalid argument");
        return RT_ERR_INVALID_ARG;
    }
    for (int i = 0; i < kMlpParams; ++i)
        if (!std::isfinite(w_host[i])) {
            set_error("rt_cache_init: non-finite weight");
            return RT_ERR_INVALID_ARG;
        }
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t* S = static_cast<uint8_t*>(state);
    std::vector<uint16_t> wb(kMlpParams);
    for (int i = 0; i < kMlpParams; ++i) {
        uint32_t u;
        std::memcpy(&u, &w_host[i], 4);
        u += 0x7fffu + ((u >> 16) & 1u);
        wb[i] = (uint16_t)(u >> 16);
    }
    HIP_TRY(hipMemsetAsync(S, 0, L.total, st));
    HIP_TRY(hipMemcpyAsync(S + L.w_master, w_host, 4 * (size_t)kMlpParams, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(S + L.w_bf16, wb.data(), 2 * (size_t)kMlpParams, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // the host staging vector goes out of scope
    return RT_OK;
}

size_t rt_render_cached_workspace_bytes(const rt_scene* scene, const rt_camera* cam, const rt_params* params,
                                        const rt_cache* cache) {
    if (!scene || !cam || !params) {
        set_error("rt_render_cached_workspace_bytes: NULL argument");
        return 0;
    }
    CachePlan cp;
    std::string why;
    if (!make_cache_plan(scene->h, *cam, *params, cache, cp, why)) {
        set_error("rt_render_cached_workspace_bytes: " + why);
        return 0;
    }
    return cp.total;
}

rt_status rt_render_cached(const rt_scene* scene, const rt_camera* cam, const rt_params* params, const rt_cache* cache,
                           float* out_rgb, int32_t* out_hit_ids) {
    if (!scene || !cam || !params || !out_rgb) {
        set_error("rt_render_cached: NULL argument");
        return RT_ERR_INVALID_ARG;
    }
    const SceneHost& h = scene->h;
    if (!h.dev) {
        set_error("rt_render_cached: scene not uploaded (call rt_scene_upload)");
        return RT_ERR_NOT_UPLOADED;
    }
    const rt_params& p = *params;
    if (!std::isfinite(p.eps) || p.eps < 0.0f || !(cam->vfov_deg > 0.0f && cam->vfov_deg < 180.0f)) {
        set_error("rt_render_cached: invalid eps or vfov");
        return RT_ERR_INVALID_ARG;
    }
    CacheArgs C;
    std::memset(&C, 0, sizeof C);
    std::string why;
    if (!make_cache_plan(h, *cam, p, cache, C.cp, why)) {
        set_error("rt_render_cached: " + why);
        return RT_ERR_INVALID_ARG;
    }
    if (C.cp.c.depth > p.max_depth) {
        set_error("rt_render_cached: cache depth must not exceed max_depth");
        return RT_ERR_INVALID_ARG;
    }
    if (!p.workspace || p.workspace_bytes < C.cp.total) {
        set_error("rt_render_cached: workspace missing or smaller than rt_render_cached_workspace_bytes (" +
                  std::to_string(C.cp.total) + ")");
        return RT_ERR_CAPACITY;
    }
    if ((reinterpret_cast<uintptr_t>(p.workspace) | reinterpret_cast<uintptr_t>(out_rgb) |
         reinterpret_cast<uintptr_t>(cache->state)) & 255) {
        set_error("rt_render_cached: device pointers must be 256-byte aligned");
        return RT_ERR_INVALID_ARG;
    }
    FrameArgs& A = C.F;
    A.sc = h.dev_view();
    camera_consts(*cam, p, A.cam);
    A.cam.frame = 0;
    for (int i = 0; i < 3; ++i) A.shc.bg[i] = p.bg[i];
    A.shc.eps = p.eps;
    A.shc.seed = p.seed;
    A.shc.max_depth = p.max_depth;
    A.shc.spp = p.spp;
    A.shc.qcap = C.cp.base.qcap;
    A.shc.scap = C.cp.base.scap;
    A.shc.per_sample = (p.flags & RT_FLAG_PER_SAMPLE) ? 1 : 0;
    A.shc.acc_off = 0;
    A.shc.out_ids = out_hit_ids;
    A.shc.gi = (p.flags & RT_FLAG_GI) ? 1 : 0;
    // depth-0 background / ambient terms summed over the four samples of a pixel in a block
    A.shc.sum_depth0 = (!A.shc.per_sample && C.cp.base.spp_pass % 4 == 0) ? 1 : 0;
    defer_and_bin_shadows(A, scene->h);
    A.pl = C.cp.base;
    A.ws = static_cast<uint8_t*>(p.workspace);
    A.shc.light_pts = scene->h.area_lights ? reinterpret_cast<const float4*>(A.ws + A.pl.off_lpts) : nullptr;
    A.stats = static_cast<rt_stats*>(p.stats);
    A.out_rgb = out_rgb;
    A.out_ids = out_hit_ids;
    A.count_work = (p.flags & RT_FLAG_COUNT_WORK) != 0;
    A.spp = p.spp;
    A.time_kernels = (p.flags & RT_FLAG_TIME_KERNELS) != 0;
    A.time_shadow = (p.flags & RT_FLAG_TIME_SHADOW) != 0;
    A.chunk = p.queue_chunk > 0 ? (uint32_t)((std::min(p.queue_chunk, 1 << 16) + 63) / 64 * 64) : 128u;
    A.tile = p.tile;
    C.state = static_cast<uint8_t*>(cache->state);
    rt_status rs = frame_grids(A);
    if (rs != RT_OK) return rs;
    hipStream_t st = static_cast<hipStream_t>(p.stream);
    HIP_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(A.ws + A.pl.off_ctr + 4 * kCtrFrame), (int)p.frame, 1,
                              st));
    HIP_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(A.ws + A.pl.off_ctr + 4 * kCtrAccum), 0, 1, st));
    // the target paths' counters carry the frame number too (it keys their random numbers)
    HIP_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(A.ws + C.cp.off_tctr + 4 * kCtrFrame), (int)p.frame, 1,
                              st));
    const bool graph = (p.flags & (RT_FLAG_NO_GRAPH | RT_FLAG_TIME_KERNELS | RT_FLAG_TIME_SHADOW)) == 0;
    rs = launch_cached(C, st, graph, h.uid);
    if (rs != RT_OK) return rs;
    if (p.flags & RT_FLAG_SYNC) {
        HIP_TRY(hipStreamSynchronize(st));
        if (A.stats) {
            uint32_t status = 0;
            HIP_TRY(hipMemcpy(&status, &A.stats->status, 4, hipMemcpyDeviceToHost));
            if (status & ~(uint32_t)RT_STATUS_CACHE_FALLBACK) {
                set_error("rt_render_cached: queue overflow (status " + std::to_string(status) + ")");
                return RT_ERR_CAPACITY;
            }
        }
    }
    return RT_OK;
}

rt_status rt_kernel_times(double* ms, int64_t* launches, int32_t reset) {
    std::lock_guard<std::mutex> g(g_time_mu);
    for (const EventPair& e : g_pending) {
        float t = 0.0f;
        HIP_TRY(hipEventSynchronize(e.b));
        HIP_TRY(hipEventElapsedTime(&t, e.a, e.b));
        g_time_ms[e.kind] += t;
        g_time_n[e.kind] += 1;
        g_event_pool.push_back(e.a);
        g_event_pool.push_back(e.b);
    }
    g_pending.clear();
    for (int k = 0; k < 5; ++k) {
        if (ms) ms[k] = g_time_ms[k];
        if (launches) launches[k] = g_time_n[k];
        if (reset) {
            g_time_ms[k] = 0.0;
            g_time_n[k] = 0;
        }
    }
    return RT_OK;
}

size_t rt_render_batch_workspace_bytes(const rt_scene* const* scenes, const rt_camera* cams, const rt_params* params,
                                       int32_t n) {
    BatchPlan bp;
    std::string why;
    if (!make_batch_plan(scenes, cams, params, n, nullptr, nullptr, bp, nullptr, why)) {
        set_error("rt_render_batch_workspace_bytes: " + why);
        return 0;
    }
    return bp.total;
}

rt_status rt_render_batch(const rt_scene* const* scenes, const rt_camera* cams, const rt_params* params, int32_t n,
                          float* const* out_rgb, int32_t* const* out_hit_ids) {
    if (!out_rgb) {
        set_error("rt_render_batch: NULL out_rgb");
        return RT_ERR_INVALID_ARG;
    }
    BatchPlan bp;
    std::string why;
    std::vector<BatchScene> table;
    if (!make_batch_plan(scenes, cams, params, n, out_rgb, out_hit_ids, bp, &table, why)) {
        set_error("rt_render_batch: " + why);
        return RT_ERR_INVALID_ARG;
    }
    const rt_params& p = params[0];
    if (!p.workspace || p.workspace_bytes < bp.total) {
        set_error("rt_render_batch: workspace missing or smaller than rt_render_batch_workspace_bytes (" +
                  std::to_string(bp.total) + ")");
        return RT_ERR_CAPACITY;
    }
    if (reinterpret_cast<uintptr_t>(p.workspace) & 255) {
        set_error("rt_render_batch: workspace must be 256-byte aligned");
        return RT_ERR_INVALID_ARG;
    }
    BatchArgs B;
    std::memset(&B, 0, sizeof B);
    B.pl = bp;
    B.ws = static_cast<uint8_t*>(p.workspace);
    B.stats = static_cast<rt_stats*>(p.stats);
    B.count_work = (p.flags & RT_FLAG_COUNT_WORK) != 0;
    B.time_kernels = (p.flags & RT_FLAG_TIME_KERNELS) != 0;
    B.time_shadow = (p.flags & RT_FLAG_TIME_SHADOW) != 0;
    B.chunk = p.queue_chunk > 0 ? (uint32_t)((std::min(p.queue_chunk, 1 << 16) + 63) / 64 * 64) : 128u;
    rt_status rs = batch_grids(B);
    if (rs != RT_OK) return rs;
    hipStream_t st = static_cast<hipStream_t>(p.stream);
    rs = upload_table(table, B.ws + bp.off_tab, st);
    if (rs != RT_OK) return rs;
    const bool graph = (p.flags & (RT_FLAG_NO_GRAPH | RT_FLAG_TIME_KERNELS | RT_FLAG_TIME_SHADOW)) == 0;
    rs = launch_batch(B, st, graph);
    if (rs != RT_OK) return rs;
    if (p.flags & RT_FLAG_SYNC) {
        HIP_TRY(hipStreamSynchronize(st));
        if (B.stats) {
            uint32_t status = 0;
            HIP_TRY(hipMemcpy(&status, &B.stats->status, 4, hipMemcpyDeviceToHost));
            if (status) {
                set_error("rt_render_batch: ray queue overflow (status " + std::to_string(status) +
                          "); raise queue_factor");
                return RT_ERR_CAPACITY;
            }
        }
    }
    return RT_OK;
}

}  // extern "C"
