/*
 * mirt.h -- C ABI of the MI355X (gfx950) Whitted ray tracer.
 *
 * Method: "Massively Parallel Ray Tracing Algorithm Using GPU" (arXiv
 * 1504.03151).  An image is made by tracing one ray per pixel and sample
 * through an image plane (Section III); each ray finds its closest object
 * (Algorithm 1's object loop), sends a shadow ray to every light (Algorithm
 * 1's blocker loop, "break" on the first blocker), and spawns reflected and
 * refracted secondary rays up to a maximum recursion depth (Section III,
 * Fig. 3), the recursion being run as iterations (Section IV.A).  Spheres
 * follow Eq. 9-12 (Section IV.B); triangles, planes, the BVH, Phong shading
 * and Fresnel-weighted dielectrics extend the paper's sphere-only scenes.
 *
 * Conventions for every entry point:
 *  - Every call returns an rt_status (0 = RT_OK, < 0 = error); C++ exceptions
 *    never cross this boundary.  rt_last_error() returns a thread-local
 *    message describing the last failure on the calling thread.
 *  - Host pointers are read during the call only.  Device pointers (scene
 *    blob, workspace, outputs, stats) are allocated and owned by the caller
 *    (e.g. with torch); the library never allocates or frees device memory.
 *  - Device pointers must be 256-byte aligned.
 *  - GPU work is enqueued on the given HIP stream (NULL = the null stream)
 *    and the call returns after enqueueing, unless RT_FLAG_SYNC is set.
 *  - Primitive ids: sphere i -> i; triangle j -> n_spheres + j; plane k ->
 *    n_spheres + n_tris + k; miss -> -1.  The BVH reorders primitives
 *    internally but every output carries the original ids.
 */
#ifndef MIRT_H
#define MIRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rt_status;
enum {
    RT_OK = 0,
    RT_ERR_INVALID_ARG = -1,    /* NULL, NaN/Inf, r <= 0, bad material index, zero sizes ... */
    RT_ERR_UNSUPPORTED = -2,    /* valid request this build does not handle */
    RT_ERR_HIP = -3,            /* a HIP runtime call failed */
    RT_ERR_BVH_DEPTH = -4,      /* BVH deeper than rt_build_opts.max_depth */
    RT_ERR_CAPACITY = -5,       /* workspace too small, or a ray queue overflowed */
    RT_ERR_DEVICE_STATUS = -6,  /* the device reported a fault in rt_stats.status */
    RT_ERR_NOT_UPLOADED = -7    /* rt_scene_upload has not been called */
};

enum { RT_MAT_PHONG = 0, RT_MAT_MIRROR = 1, RT_MAT_DIELECTRIC = 2 };

/* Phong reflection model: local = k_a*albedo + sum over unblocked lights of
 * I * (k_d*albedo*max(N.L,0) + k_s*max(R.V,0)^shininess), R the mirror
 * direction of L (Phong, not Blinn).  PHONG and MIRROR add k_r * (reflected
 * radiance); DIELECTRIC adds F * reflected + (1-F) * transmitted radiance with
 * Schlick's F and index of refraction ior (air outside). 40 bytes. */
typedef struct {
    float albedo[3];
    float k_a, k_d, k_s, shininess, k_r, ior;
    int32_t type;
} rt_material;

enum { RT_LIGHT_POINT = 0, RT_LIGHT_PARALLELOGRAM = 1, RT_LIGHT_DISK = 2 };
/* A light.  A point light sits at pos.  An area light is sampled at one point
 * per pass (frame, sample index) for every pixel, the paper's progressive
 * scheme (Section V): the parallelogram pos + a u + b v, or the ellipse (disk)
 * pos + sqrt(a) (cos(2 pi b) u + sin(2 pi b) v), with (a, b) the PCG hash
 * values of the camera jitter taken with the pixel slot 0xFFFFFFFF - (light
 * index); the sample point then acts as a point light of this intensity. */
typedef struct {
    float pos[3];
    float intensity[3];
    int32_t shape;               /* RT_LIGHT_* */
    float u[3], v[3];            /* area lights: edge or semi-axis vectors (ignored for points) */
} rt_light;

/* Scene arrays (host memory, copied by rt_build_scene). */
typedef struct {
    const float* spheres;        /* [n_spheres][4]  cx, cy, cz, r (r > 0) */
    int64_t n_spheres;
    const int32_t* sphere_mat;   /* [n_spheres] material index */
    const float* tris;           /* [n_tris][3][3]  vertices, counter-clockwise seen from outside */
    int64_t n_tris;
    const int32_t* tri_mat;      /* [n_tris] */
    const float* planes;         /* [n_planes][4]  nx, ny, nz, h with n.x = h, |n| = 1 */
    int64_t n_planes;
    const int32_t* plane_mat;    /* [n_planes] */
    const rt_material* materials;
    int32_t n_materials;
    const rt_light* lights;      /* point and area lights */
    int32_t n_lights;
} rt_scene_desc;

enum { RT_LAYOUT_DFS = 0, RT_LAYOUT_BFS = 1, RT_LAYOUT_TREELET = 2, RT_LAYOUT_BVH4 = 3, RT_LAYOUT_BVH4Q = 4 };

/* BVH build options; zero fields take the defaults in brackets. */
typedef struct {
    int32_t leaf_max;     /* [4]  split while a node holds more primitives (<= 15) */
    int32_t sah_bins;     /* [32] centroid bins per axis of the binned SAH build */
    int32_t max_depth;    /* [60] deeper trees fail with RT_ERR_BVH_DEPTH (<= 61: LDS stack budget) */
    int32_t node_layout;  /* [0]  order of the 64-byte nodes in memory (root first in every layout):
                             RT_LAYOUT_DFS depth-first pre-order (left child at index + 1),
                             RT_LAYOUT_BFS breadth-first (level by level),
                             RT_LAYOUT_TREELET blocks of up to 7 nodes (three levels of a subtree,
                             breadth-first inside) stored contiguously, blocks in depth-first order,
                             RT_LAYOUT_BVH4 the binary tree collapsed into 128-byte four-wide nodes
                             (depth-first), RT_LAYOUT_BVH4Q the same tree in 64-byte nodes whose child
                             boxes are 8-bit codes on a power-of-two grid per axis, rounded outward;
                             RT_ERR_BVH_DEPTH if a four-wide traversal stack would exceed 96 */
} rt_build_opts;

/* Pinhole camera: vfov_deg is the vertical field of view; pixel row 0 is the
 * top row; right = normalize(up x forward); pixel (px, py), sample offset
 * (jx, jy) in [0,1)^2 looks along normalize(f + X r + Y u) with
 * X = (2 (px + jx) / W - 1) (W / H) tan(vfov/2), Y = (1 - 2 (py + jy) / H) tan(vfov/2). */
typedef struct {
    float eye[3], look_at[3], up[3];
    float vfov_deg;
    int32_t width, height;
} rt_camera;

enum {
    RT_FLAG_SYNC = 1,        /* synchronize the stream and check rt_stats.status before returning */
    RT_FLAG_COUNT_WORK = 2,  /* count BVH node visits and primitive tests into rt_stats (slower) */
    RT_FLAG_NO_GRAPH = 4,    /* launch kernels one by one instead of replaying a captured HIP graph */
    RT_FLAG_TIME_KERNELS = 8, /* record HIP events around every traversal and shading launch on the
                                 frame's stream (implies RT_FLAG_NO_GRAPH); read with rt_kernel_times */
    RT_FLAG_PER_SAMPLE = 16,  /* keep every sample: out_rgb is [H][W][spp][3], not averaged */
    RT_FLAG_ACCUMULATE = 32,  /* progressive rendering (rt_render only): add this frame to the accumulator
                                 left in the workspace by the previous rt_params.accum_frames frames (0: start
                                 afresh) and output the average over all of them, the paper's pass-by-pass
                                 image update (Section V) */
    RT_FLAG_GI = 64,          /* diffuse global illumination (Eq. 8, the hemisphere integral of Section II) by
                                 path tracing (rt_render and rt_render_batch; per scene in a batch): every
                                 hit still adds its Phong local terms through shadow rays, and the path
                                 continues with ONE ray while depth < max_depth, chosen at random among the
                                 diffuse bounce (weight k_d * albedo: a Lambertian BRDF k_d * albedo / pi,
                                 cosine-weighted direction normalize(N_f + s), s uniform on the unit sphere),
                                 the mirror reflection (k_r, or F for a dielectric) and the refraction
                                 (1 - F), each with probability proportional to the largest channel of its
                                 weight, and weighted by weight / probability.  Random numbers: the PCG hash
                                 chain of the camera jitter through (seed, frame, pixel), then the sample,
                                 then the word 0x80000000 | depth << 2 | k (k = 0 branch, 1 and 2 the
                                 direction); 24 bits each.  rt_render_cached: the image's paths
                                 end at the cache depth; the training targets are paths from the
                                 selected queries keyed by (training index, sample 0). */
    RT_FLAG_TIME_SHADOW = 128 /* record HIP events around the shadow traversal launches only (implies
                                 RT_FLAG_NO_GRAPH): each recorded event leaves the GPU idle for a few
                                 microseconds, so a timed frame records only the pair it needs */
};

enum { RT_TILE_8X8 = 0, RT_TILE_16X4 = 1, RT_TILE_32X2 = 2, RT_TILE_4X16 = 3 };

/* Per-frame rendering parameters. */
typedef struct {
    int32_t spp;              /* samples per pixel (>= 1); a square count is stratified */
    int32_t max_depth;        /* secondary rays spawn while depth < max_depth; primary = depth 0 (<= 15) */
    int32_t jitter;           /* 0: sample centres; 1: jitter from the PCG hash of (seed, frame, pixel, sample) */
    uint32_t frame;
    uint64_t seed;
    float bg[3];              /* radiance of rays that miss */
    float eps;                /* origin offset of spawned rays: eps * max(1, max|x_i|) along the normal */
    int32_t samples_per_pass; /* samples traced per wavefront pass; 0 = chosen from the workspace */
    int32_t flags;            /* RT_FLAG_* */
    float queue_factor;       /* ray-queue capacity per pass, in primary rays (0 = 2.0) */
    int32_t queue_chunk;      /* queue entries a traversal wave takes per fetch (0 = 128; multiple of 64) */
    int32_t tile;             /* pixels of one wave's primary rays: RT_TILE_8X8 (0), RT_TILE_16X4,
                                 RT_TILE_32X2, RT_TILE_4X16 */
    uint32_t accum_frames;    /* with RT_FLAG_ACCUMULATE: frames already in the workspace's accumulator */
    void* workspace;          /* device, rt_render_workspace_bytes() bytes */
    size_t workspace_bytes;
    void* stats;              /* device rt_stats or NULL; accumulated, caller zeroes it */
    void* stream;             /* hipStream_t */
} rt_params;

#define RT_STATS_MAX_DEPTH 16
/* Bits of rt_stats.status.  The first three are faults (rays were dropped; a
 * frame with RT_FLAG_SYNC returns RT_ERR_CAPACITY); RT_STATUS_CACHE_FALLBACK
 * is a report: a learned-form frame found its cache state unhealthy and was
 * rendered by the plain tracer instead (see rt_render_cached). */
enum {
    RT_STATUS_RAY_OVERFLOW = 1,      /* a closest-hit ray queue overflowed */
    RT_STATUS_SHADOW_OVERFLOW = 2,   /* a shadow queue overflowed */
    RT_STATUS_CACHE_RECORDS = 4,     /* the learned form's query records overflowed */
    RT_STATUS_CACHE_FALLBACK = 8     /* the learned form fell back to the plain tracer */
};
/* Device-side counters, accumulated by rt_render (caller zeroes them). */
typedef struct {
    uint32_t status;          /* RT_STATUS_* bits */
    uint32_t passes;
    uint64_t rays[RT_STATS_MAX_DEPTH];    /* closest-hit queries issued per depth */
    uint64_t shadow[RT_STATS_MAX_DEPTH];  /* shadow (any-hit) queries issued per depth */
    uint64_t node_visits;     /* with RT_FLAG_COUNT_WORK: BVH nodes fetched by closest-hit queries */
    uint64_t tri_tests;       /* ... ray/triangle tests of closest-hit queries */
    uint64_t sphere_tests;    /* ... ray/sphere tests of closest-hit queries */
    uint64_t shadow_node_visits, shadow_tri_tests, shadow_sphere_tests;
    uint64_t cache_queries;   /* learned form: network queries (hits at the cache depth) */
    uint64_t target_rays;     /* learned form: closest-hit queries traced for training targets */
    uint64_t target_shadow;   /* ... and their shadow queries (not counted in rays / shadow) */
} rt_stats;

typedef struct rt_scene rt_scene;   /* opaque, host memory only */

typedef struct {
    int64_t n_nodes;
    int32_t depth;          /* BVH depth (root = 0) */
    int32_t stack_size;     /* traversal stack entries a ray needs */
    int64_t n_leaves;
    int64_t n_bvh_prims;    /* spheres + triangles */
    double sah_cost;
    double build_seconds;
    float bounds_lo[3], bounds_hi[3];   /* scene bounds (spheres and triangles) */
    int32_t node_layout;    /* RT_LAYOUT_* of the nodes */
} rt_scene_info;

/* Validate the description, build a binned-SAH binary BVH over spheres and
 * triangles (planes stay in a list), pack 64-byte nodes and 48-byte leaf-order
 * primitive records.  Copies all inputs.  Errors: RT_ERR_INVALID_ARG (NULL
 * arrays with non-zero counts, non-finite values, r <= 0, |plane n| not 1,
 * material index out of range, n_lights < 0), RT_ERR_BVH_DEPTH. */
rt_status rt_build_scene(const rt_scene_desc* desc, const rt_build_opts* opts, rt_scene** out);
void rt_destroy_scene(rt_scene* scene);
rt_status rt_scene_get_info(const rt_scene* scene, rt_scene_info* out);
/* Re-lay the nodes of a built scene in another RT_LAYOUT_* (the same binary
 * tree, or its four-wide collapse; every query returns the same hit).  Drops
 * the scene's device copy and may change rt_scene_device_bytes and the
 * workspace size: call rt_scene_upload again before rendering.  Errors:
 * RT_ERR_INVALID_ARG (NULL scene, unknown layout), RT_ERR_BVH_DEPTH. */
rt_status rt_scene_set_layout(rt_scene* scene, int32_t node_layout);

/* Bytes of the device blob (nodes | primitives | normals | planes | materials | lights | refit order). */
size_t rt_scene_device_bytes(const rt_scene* scene);
/* Copy the blob into caller-owned device memory dev_ptr (>= rt_scene_device_bytes)
 * on stream; the scene keeps dev_ptr, which must stay valid while it is used. */
rt_status rt_scene_upload(rt_scene* scene, void* dev_ptr, size_t bytes, void* stream);

/* BVH refit on the GPU, for dynamic scenes (moving primitives, same tree; the
 * acceleration structure of Section II kept valid without a host rebuild).
 * spheres: device float [n_spheres][4] (centre, radius) and tris: device float
 * [n_tris][3][3], the scene's primitives in the order it was built with (NULL
 * when the count is 0); materials, planes and lights are kept.  Enqueued on
 * stream: rewrites the uploaded blob's primitive records and triangle normals,
 * then the child boxes of every node level by level from the deepest (any
 * node layout; quantized nodes are requantized), with the build's outward
 * padding from the new scene scale.  Refitting to the positions the scene was
 * built with reproduces the uploaded blob bit for bit.  The tree's quality
 * falls as primitives move from where it was built (more node visits, never a
 * wrong hit).  workspace: device, >= rt_scene_refit_workspace_bytes (a box per
 * node), 256-byte aligned; not shared with a concurrent call.  Only the device
 * copy changes: rt_scene_upload, rt_scene_set_layout, rt_host_trace and
 * rt_scene_get_info keep the geometry the scene was built with.  With
 * RT_FLAG_SYNC in flags the call waits and returns RT_ERR_INVALID_ARG if a
 * position is non-finite or a radius <= 0 (the kernels then change nothing);
 * without it such input is skipped the same way but not reported.  Errors:
 * RT_ERR_INVALID_ARG, RT_ERR_NOT_UPLOADED, RT_ERR_CAPACITY, RT_ERR_HIP. */
size_t rt_scene_refit_workspace_bytes(const rt_scene* scene);
rt_status rt_scene_refit(rt_scene* scene, const float* spheres, const float* tris, void* workspace,
                         size_t workspace_bytes, int32_t flags, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight per-frame loops of dynamic scenes, harnesses that forbid
 * hipMalloc): rt_scene_refit with its scratch (the refit header and a box per
 * node, rt_scene_refit_workspace_bytes) taken from a buffer the library holds
 * in static device memory, at most rt_scene_refit_noalloc_max_bytes() (32 MiB:
 * up to 1,398,090 nodes) per GPU, kept until the process ends.  Same kernels,
 * same results, same flags and errors as rt_scene_refit, plus RT_ERR_CAPACITY
 * for a scene whose scratch exceeds the maximum.  Allocates nothing: no
 * hipMalloc, hipFree or allocating library call.  All calls on one GPU share
 * the buffer: calls that overlap on one GPU (two streams, two threads) race
 * and must be ordered by the caller. */
size_t rt_scene_refit_noalloc_max_bytes(void);
rt_status rt_scene_refit_noalloc(rt_scene* scene, const float* spheres, const float* tris, int32_t flags,
                                 void* stream);

/* Workspace bytes rt_render needs for this camera and parameters (queues,
 * accumulator, counters).  Returns 0 and sets the last error for invalid input. */
size_t rt_render_workspace_bytes(const rt_scene* scene, const rt_camera* cam, const rt_params* params);

/* Render one frame.  out_rgb: device float [H][W][3], linear radiance averaged
 * over spp (no clamp, no gamma).  out_hit_ids: device int32 [H][W][spp], the
 * original id of each primary ray's closest hit (-1 miss), or NULL. */
rt_status rt_render(const rt_scene* scene, const rt_camera* cam, const rt_params* params, float* out_rgb,
                    int32_t* out_hit_ids);

/* Render n scenes in one batched wavefront (one queue shared by all scenes).
 * cams[i], params[i] as for rt_render except that workspace, stats, stream and
 * flags are taken from params[0]; workspace from rt_render_batch_workspace_bytes. */
size_t rt_render_batch_workspace_bytes(const rt_scene* const* scenes, const rt_camera* cams,
                                       const rt_params* params, int32_t n);
rt_status rt_render_batch(const rt_scene* const* scenes, const rt_camera* cams, const rt_params* params,
                          int32_t n, float* const* out_rgb, int32_t* const* out_hit_ids);

/* Closest hit of n arbitrary rays: Algorithm 1's object loop (the nearest
 * object along the ray), through the BVH; spheres by Eq. 9-12.  rays: device
 * float [n][8] = ox, oy, oz, dx, dy, dz (unit length), tmin (ignored, the
 * range is (0, tmax)), tmax (<= 0 or inf: unbounded).  Outputs (device): t [n]
 * (inf on a miss), id [n] original ids (-1 miss), and uv [n][2] (NULL: not
 * written; 8-byte aligned) the hit's surface coordinates: for a triangle the
 * barycentric weights (u, v) of its second and third vertex (hit point =
 * (1-u-v) v0 + u v1 + v v2); for a sphere the outward normal n at the hit in
 * spherical coordinates, u = (atan2(n_z, n_x) + pi) / (2 pi), v = acos(n_y) / pi;
 * (0, 0) for planes and misses.  workspace: device, >= 64 bytes (counters).
 * Errors: RT_ERR_INVALID_ARG (NULL buffers with n > 0, misaligned uv),
 * RT_ERR_NOT_UPLOADED, RT_ERR_UNSUPPORTED (traversal stack beyond LDS). */
rt_status rt_intersect(const rt_scene* scene, const float* rays, int64_t n, float* t, int32_t* id, float* uv,
                       void* workspace, void* stream);
/* Any hit in (0, tmax) of n rays: Algorithm 1's blocker loop for shadow rays,
 * which stops at the first blocker (same layout; tmax must be finite and > 0);
 * occluded [n] device uint8 (1 = blocked). */
rt_status rt_occluded(const rt_scene* scene, const float* rays, int64_t n, uint8_t* occluded, void* workspace,
                      void* stream);

/* Host FP32 traversal of the same packed BVH (the fair CPU comparison and the
 * source of per-ray work counts).  rays, t, id, work are HOST arrays; work
 * [n][3] (node visits, triangle tests, sphere tests) may be NULL.
 * any_hit = 1 answers the shadow query (id = hit or -1). nthreads <= 0: all cores. */
rt_status rt_host_trace(const rt_scene* scene, const float* rays, int64_t n, int32_t any_hit, float* t,
                        int32_t* id, uint32_t* work, int32_t nthreads);

/* Kernel timings recorded by frames rendered with RT_FLAG_TIME_KERNELS (or
 * RT_FLAG_TIME_SHADOW, which records index 2 only) since the last reset: total milliseconds and launch counts of the closest-hit
 * (index 0), shading (1) and shadow any-hit (2) kernels, the cache inference
 * (3) and a learned frame's whole training part (4).  Waits for the recorded
 * events.  ms [5] and launches [5] are host arrays; reset != 0 clears the
 * totals after reading. */
rt_status rt_kernel_times(double* ms, int64_t* launches, int32_t reset);

/* ---- radiance-cache network (BF16 operands on the matrix cores, FP32 accumulation) ----
 * A small MLP that stands in for the radiance of rays below bounce 2 (the
 * learned form of the recursive step).  Input: 64 features (the 36 sin/cos
 * frequency encodings of the hit position normalised to the scene bounds,
 * the facing normal and the view direction, zero-padded from 42); five hidden
 * layers of 64 with ReLU; 3 outputs; no biases.  Weights are row-major
 * (out, in): W1..W5 [64][64] then W6 [3][64] = rt_mlp_num_params() values.
 * Every pointer below is a device pointer; BF16 values are uint16 bit patterns.
 * w_bf16 and x_bf16 must be 16-byte aligned (RT_ERR_INVALID_ARG otherwise). */
int32_t rt_mlp_num_params(void);
/* y [n][3] = network(x_bf16 [n][64]). */
rt_status rt_mlp_forward(const uint16_t* w_bf16, const uint16_t* x_bf16, int64_t n, float* y, void* stream);
/* Relative-L2 loss mean((y - t)^2 / (y^2 + 0.01)) over n_total samples: adds
 * this batch's weight gradients into dw [num_params] (FP32) and its summed
 * per-sample loss terms into loss_sum [1]. */
rt_status rt_mlp_grad(const uint16_t* w_bf16, const uint16_t* x_bf16, const float* target, int64_t n,
                      int64_t n_total, float* dw, float* loss_sum, void* stream);
/* One Adam step (step >= 1, bias-corrected) on FP32 master weights w; refreshes
 * w_bf16 and clears grad. */
rt_status rt_mlp_adam(float* w, uint16_t* w_bf16, float* m, float* v, float* grad, int32_t step, float lr,
                      float b1, float b2, float eps, void* stream);

/* ---- learned form: frames whose recursion below `depth` is answered by the network ----
 * At depth `depth`, a ray that misses returns the background and a ray that
 * hits adds w * max(network(features(x, N_f, V)), 0) instead of its local
 * shading and recursion.  With RT_CACHE_TRAIN the frame also picks up to
 * train_samples of these queries (stratified, random per-frame offset), traces
 * their rays on to full_depth with the plain tracer (the training targets)
 * and takes train_steps Adam steps on the relative-L2 loss.  The image uses
 * the weights from before the frame's training.
 *
 * Health and fallback (the plain tracer is the learned form's fallback): after
 * a frame's training steps the library checks the loss sums, the FP32 master
 * weights and the Adam moments, and at the start of every learned-form frame
 * the BF16 weights it is about to use; any non-finite value sets a health bit
 * in the state.  A frame that starts with a health bit set answers no query:
 * its hits at `depth` are shaded and traced on to params->max_depth by the
 * plain tracer on the device (no host round trip), so the image is the plain
 * frame's, and rt_stats.status reports RT_STATUS_CACHE_FALLBACK.  The bits
 * stay set until rt_cache_init initialises the state again.  A healthy frame
 * pays for the fallback chain's empty launches only (tens of microseconds). */
enum { RT_CACHE_INFER = 1, RT_CACHE_TRAIN = 2 };
enum {
    RT_CACHE_HEALTH_LOSS = 1,        /* a training step's loss sum was not finite */
    RT_CACHE_HEALTH_WEIGHTS = 2,     /* a master weight or Adam moment was not finite after training */
    RT_CACHE_HEALTH_BF16 = 4         /* a BF16 weight was not finite at the start of a frame */
};
typedef struct {
    int32_t mode;              /* RT_CACHE_INFER or RT_CACHE_TRAIN */
    int32_t depth;             /* [2] depth whose hits query the network (>= 1) */
    int32_t full_depth;        /* [8] recursion depth of the training targets */
    int32_t train_samples;     /* [65536] queries trained on per frame (<= the state's capacity) */
    int32_t train_steps;       /* [4] Adam steps per frame, on equal slices of the samples */
    float lr, b1, b2, eps;     /* [1e-3, 0.9, 0.999, 1e-8] */
    float bounds_lo[3], bounds_hi[3];   /* encoding bounds; all zero: the scene's bounds */
    void* state;               /* device, rt_cache_state_bytes(capacity) bytes, set up by rt_cache_init */
} rt_cache;

/* Byte offsets inside the cache state.  counters (uint32): [0] Adam steps
 * taken, [1] training samples of the last frame, [2..17] the last frame's
 * per-step loss sums (float bits; divide by 3 x slice size), [18] health bits
 * (RT_CACHE_HEALTH_*; 0 = healthy).  The last
 * frame's training batch: train_rays [cap][6] (o, d at the cache depth),
 * train_feats [cap][64] BF16, train_targets [cap][3], train_pix [cap]
 * (accumulation slot of each sample's pixel). */
typedef struct {
    size_t w_master, w_bf16, m, v, grad, counters, train_rays, train_feats, train_targets, train_pix, total;
    int32_t capacity;
} rt_cache_layout;
rt_status rt_cache_state_layout(int32_t capacity, rt_cache_layout* out);
size_t rt_cache_state_bytes(int32_t capacity);
/* Initialise a state: FP32 master weights from w_host [rt_mlp_num_params()] (host), their
 * BF16 copy, zero moments, gradients and counters. */
rt_status rt_cache_init(void* state, int32_t capacity, const float* w_host, void* stream);
size_t rt_render_cached_workspace_bytes(const rt_scene* scene, const rt_camera* cam, const rt_params* params,
                                        const rt_cache* cache);
/* One learned-form frame (all samples in one pass); arguments as rt_render. */
rt_status rt_render_cached(const rt_scene* scene, const rt_camera* cam, const rt_params* params,
                           const rt_cache* cache, float* out_rgb, int32_t* out_hit_ids);

const char* rt_last_error(void);
const char* rt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MIRT_H */
