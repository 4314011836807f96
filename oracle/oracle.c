/*
 * oracle.c -- FP64 reference Whitted ray tracer.  TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, brute-force statement of what the GPU ray
 * tracer computes.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product library never does, and the two
 * share no code (no headers, no helpers, no tables).
 *
 * What it computes (paper: "Massively Parallel Ray Tracing Algorithm Using
 * GPU", arXiv 1504.03151):
 *   - Closest hit by brute force over every primitive: the object loop of
 *     Algorithm 1 (Section III).  No acceleration structure.
 *   - Sphere hits from the quadratic of Eq. 11-12 (Section IV.B), taking the
 *     smallest root in (0, tmax) (the paper does not say which root).
 *   - Triangles by an edge-function test in FP64 (inclusive edges, zero-area
 *     never hit); planes by the plane equation.
 *   - Shadow rays to each light (a point light, or the pass's sample point of an
 *     area light), counted as blocked by the first
 *     primitive found on the segment: the inner loop of Algorithm 1 with its
 *     ELSE branch read as "add the light's term only if nothing blocks".
 *   - Recursion over reflected and refracted secondary rays up to a maximum
 *     depth (Section III after Algorithm 1, Section IV.A, Fig. 3), with the
 *     local term from Phong reflection (ambient + diffuse + specular) in place
 *     of the hemisphere integral of Eq. 8.
 *   - Several samples per pixel averaged (anti-aliasing, end of Section III).
 *   - Optionally (or_params.gi) diffuse global illumination: the hemisphere
 *     integral of Eq. 8 estimated by path tracing, one randomly chosen
 *     continuation per hit (see gi_bounce).
 *
 * Besides colours and ids it reports, for every ray it traces, a robustness
 * margin: how far each discrete decision (which primitive is hit, whether a
 * shadow ray is blocked, whether the ray is inside a dielectric, total
 * internal reflection) is from flipping.  It combines
 *   (a) relative margins: barycentric min(lambda) for triangles,
 *       1-(d_perp/r)^2 for spheres, |n.d| for planes, (t2-t1)/t1 for depth
 *       ties, |t|/max(1,|o|) and |tmax-t|/tmax for the ends of the segment;
 *   (b) 1e-4 x (world-space clearance / FP32 error envelope), where the
 *       envelope is propagated along the ray tree (curved mirrors and
 *       refraction amplify round-off of the FP32 implementation).
 * margin = min over all decisions; a ray is robust when margin > 1e-4.
 * Rays that are not robust may legitimately differ between an FP32 and an
 * FP64 implementation.  A sample (pixel) is robust when every decision of its
 * ray tree that can move its radiance by more than 1e-4 is robust; decisions
 * below that effect (deep, low-weight rays), up to 3e-4 in total per sample,
 * cannot break a 1e-3 RGB comparison and are left out of its margin.  The
 * per-ray margins (or_closest, or_occluded, the ray log) are never relaxed.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -o liboracle.so oracle.c -lm -lpthread
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define OR_INF (1.0 / 0.0)
/* FP32 arithmetic error allowance, relative to coordinate magnitude (~7 ulp). */
#define EA 4e-7
/* Margins are reported capped at this value: above it they are irrelevant
 * for the 1e-4 robustness threshold. */
#define MARGIN_CAP 1e-2

enum { MAT_PHONG = 0, MAT_MIRROR = 1, MAT_DIELECTRIC = 2 };

typedef struct {
    int64_t n_spheres;
    const float* spheres;     /* [n][4] cx cy cz r */
    const int32_t* sphere_mat;
    int64_t n_tris;
    const float* tris;        /* [n][3][3] */
    const int32_t* tri_mat;
    int64_t n_planes;
    const float* planes;      /* [n][4] nx ny nz h : n.x = h */
    const int32_t* plane_mat;
    int32_t n_materials;
    const float* materials;   /* [m][10] albedo rgb, ka, kd, ks, shininess, kr, ior, type */
    int32_t n_lights;
    const float* lights;      /* [l][13] pos, intensity, shape, u, v (see or_light_point) */
} or_scene;

#define LW 13   /* floats per light */

typedef struct {
    double eye[3], look_at[3], up[3];
    double vfov_deg;
    int32_t width, height;
} or_camera;

typedef struct {
    int32_t spp, max_depth, jitter;
    int32_t gi;       /* 1: diffuse global illumination by path tracing (see trace) */
    uint64_t seed;
    uint32_t frame, pad1;
    double bg[3];
    double eps;
} or_params;

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                     */
/* ------------------------------------------------------------------------ */
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(double* r, const double* a, const double* b) { r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2]; }
static void cross3(double* r, const double* a, const double* b) {
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    r[0] = x; r[1] = y; r[2] = z;
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }
static void normalize3(double* a) { double n = norm3(a); a[0] /= n; a[1] /= n; a[2] /= n; }
static double maxabs3(const double* a) { return fmax(fabs(a[0]), fmax(fabs(a[1]), fabs(a[2]))); }
static void load3f(double* r, const float* f) { r[0] = f[0]; r[1] = f[1]; r[2] = f[2]; }

/* ------------------------------------------------------------------------ */
/* counter-based hash for pixel jitter: the 32-bit PCG hash of Jarzynski and */
/* Olano, "Hash Functions for GPU Rendering", JCGT 9(3), 2020 (after         */
/* O'Neill's PCG generator).                                                 */
/* ------------------------------------------------------------------------ */
uint32_t or_pcg(uint32_t v) {
    uint32_t state = v * 747796405u + 2891336453u;
    uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

/* xi in [0,1): 24 random bits, exact in FP32 and FP64 */
double or_jitter(uint64_t seed, uint32_t frame, uint32_t pixel, uint32_t s, uint32_t dim) {
    uint32_t h = or_pcg((uint32_t)seed);
    h = or_pcg(h ^ (uint32_t)(seed >> 32));
    h = or_pcg(h ^ frame);
    h = or_pcg(h ^ pixel);
    h = or_pcg(h ^ (s * 2u + dim));
    return (double)(h >> 8) * (1.0 / 16777216.0);
}

/* Random numbers of a path: number k of the bounce at depth `depth` of sample
 * s of a pixel.  The camera-jitter hash chain through the pixel, then the
 * sample and a word with the top bit set (no camera-jitter word has it) that
 * holds depth and k.  24 random bits, exact in FP32 and FP64. */
double or_path_rand(uint64_t seed, uint32_t frame, uint32_t pixel, uint32_t s, uint32_t depth, uint32_t k) {
    uint32_t h = or_pcg((uint32_t)seed);
    h = or_pcg(h ^ (uint32_t)(seed >> 32));
    h = or_pcg(h ^ frame);
    h = or_pcg(h ^ pixel);
    h = or_pcg(h ^ s);
    h = or_pcg(h ^ (0x80000000u | (depth << 2) | k));
    return (double)(h >> 8) * (1.0 / 16777216.0);
}

/* Light sample point.  Following the paper's progressive scheme (Section V:
 * each pass samples every light source once, and the passes add up), light l
 * is sampled at one point per (frame, sample) for all pixels:
 *   shape 0: a point light at pos;
 *   shape 1: the parallelogram pos + a u + b v;
 *   shape 2: the ellipse (disk) pos + sqrt(a) (cos(2 pi b) u + sin(2 pi b) v),
 *            uniform in area;
 * with a, b the hash values of the camera jitter taken with the pixel slot
 * 0xFFFFFFFF - l (no pixel index reaches it).  Computed in FP64 and rounded
 * once to FP32, the precision the scene's light records have. */
void or_light_point(const float* L, uint64_t seed, uint32_t frame, int32_t s, int32_t l, double* out) {
    const int shape = (int)L[6];
    if (shape == 0) {
        load3f(out, L);
        return;
    }
    const double a = or_jitter(seed, frame, 0xFFFFFFFFu - (uint32_t)l, (uint32_t)s, 0);
    const double b = or_jitter(seed, frame, 0xFFFFFFFFu - (uint32_t)l, (uint32_t)s, 1);
    double cu, cv;
    if (shape == 1) {
        cu = a;
        cv = b;
    } else {
        const double r = sqrt(a), phi = 2.0 * M_PI * b;
        cu = r * cos(phi);
        cv = r * sin(phi);
    }
    for (int i = 0; i < 3; ++i) out[i] = (double)(float)((double)L[i] + cu * (double)L[7 + i] + cv * (double)L[10 + i]);
}

/* Pinhole camera: vertical field of view, row 0 at the top, right = up x forward. */
void or_camera_ray(const or_camera* cam, const or_params* p, int64_t pixel, int32_t s, double* o, double* d) {
    double f[3], r[3], u[3];
    sub3(f, cam->look_at, cam->eye);
    normalize3(f);
    cross3(r, cam->up, f);
    normalize3(r);
    cross3(u, f, r);
    const int W = cam->width, H = cam->height;
    const int64_t px = pixel % W, py = pixel / W;
    double jx = 0.5, jy = 0.5;
    const int spp = p->spp;
    int m = (int)floor(sqrt((double)spp) + 0.5);
    double xi0 = 0.5, xi1 = 0.5;
    if (p->jitter) {
        xi0 = or_jitter(p->seed, p->frame, (uint32_t)pixel, (uint32_t)s, 0);
        xi1 = or_jitter(p->seed, p->frame, (uint32_t)pixel, (uint32_t)s, 1);
    }
    if (spp > 1 && m * m == spp) {
        jx = ((double)(s % m) + xi0) / m;
        jy = ((double)(s / m) + xi1) / m;
    } else {
        jx = xi0;
        jy = xi1;
    }
    const double th = tan(cam->vfov_deg * 0.5 * M_PI / 180.0);
    const double X = (2.0 * ((double)px + jx) / W - 1.0) * ((double)W / H) * th;
    const double Y = (1.0 - 2.0 * ((double)py + jy) / H) * th;
    for (int i = 0; i < 3; ++i) {
        o[i] = cam->eye[i];
        d[i] = f[i] + X * r[i] + Y * u[i];
    }
    normalize3(d);
}

/* ------------------------------------------------------------------------ */
/* rays and error envelopes                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    double o[3], d[3];
    double tmax;
    double so;   /* origin uncertainty of an FP32 implementation (world units) */
    double sd;   /* direction uncertainty (radians) */
} oray;

/* world-space uncertainty of the point o + t d */
static double envelope(const oray* r, double t) {
    double tt = fabs(t);
    if (!isfinite(tt)) tt = 1e30;
    return r->so + r->sd * tt + EA * (maxabs3(r->o) + tt) + 1e-30;
}

/* One primitive evaluated against one ray. */
typedef struct {
    int ok;          /* passes the shape test */
    int nroot;       /* roots (ascending) when ok */
    double t[2];
    double cs[2];    /* |cos| between ray and surface normal at each root */
    double rel;      /* signed relative shape margin (>= 0 when ok) */
    double clr;      /* signed world clearance perpendicular to the ray */
    double tref;     /* ray parameter at which the shape decision is taken */
    int valid;       /* 0: primitive can never be hit (degenerate or parallel) */
} cand;

/* Sphere: the quadratic of Eq. 11, roots by Eq. 12 with a = d.d, b = 2(o-c).d,
 * c' = (o-c).(o-c) - r^2 (the paper's c is renamed c' to keep c for the centre). */
static void eval_sphere(const float* s, const oray* ray, cand* c) {
    double ctr[3], f[3];
    load3f(ctr, s);
    const double r = s[3];
    sub3(f, ray->o, ctr);
    const double a = dot3(ray->d, ray->d);
    const double b = 2.0 * dot3(f, ray->d);
    const double cc = dot3(f, f) - r * r;
    const double disc = b * b - 4.0 * a * cc;
    const double fd = dot3(f, ray->d);
    double dp2 = dot3(f, f) - fd * fd / a;
    if (dp2 < 0) dp2 = 0;
    const double dp = sqrt(dp2);
    c->valid = 1;
    c->rel = 1.0 - dp2 / (r * r);
    c->clr = r - dp;
    c->tref = -b / (2.0 * a);
    c->ok = disc >= 0.0;
    c->nroot = 0;
    if (c->ok) {
        const double sq = sqrt(disc);
        c->t[0] = (-b - sq) / (2.0 * a);
        c->t[1] = (-b + sq) / (2.0 * a);
        c->nroot = 2;
        const double dl = sqrt(a);
        for (int i = 0; i < 2; ++i) {
            double p[3], n[3];
            for (int k = 0; k < 3; ++k) p[k] = ray->o[k] + c->t[i] * ray->d[k];
            sub3(n, p, ctr);
            c->cs[i] = fabs(dot3(n, ray->d)) / (r * dl);
        }
    }
}

/* Triangle: plane distance, then the three edge functions (barycentrics)
 * computed from cross products at the plane point; edges inclusive. */
static void eval_tri(const float* tv, const oray* ray, cand* c) {
    double v0[3], v1[3], v2[3], e1[3], e2[3], n[3];
    load3f(v0, tv);
    load3f(v1, tv + 3);
    load3f(v2, tv + 6);
    sub3(e1, v1, v0);
    sub3(e2, v2, v0);
    cross3(n, e1, e2);
    const double nn = dot3(n, n);
    const double denom = dot3(n, ray->d);
    c->valid = 0;
    c->ok = 0;
    c->nroot = 0;
    if (nn == 0.0 || denom == 0.0) return;
    c->valid = 1;
    double w[3];
    sub3(w, v0, ray->o);
    const double t = dot3(n, w) / denom;
    double p[3], a[3], b[3], q[3], lam[3];
    for (int k = 0; k < 3; ++k) p[k] = ray->o[k] + t * ray->d[k];
    const double* V[3] = {v0, v1, v2};
    double elen[3];
    for (int i = 0; i < 3; ++i) {
        const double* A = V[(i + 1) % 3];
        const double* B = V[(i + 2) % 3];
        sub3(a, A, p);
        sub3(b, B, p);
        cross3(q, a, b);
        lam[i] = dot3(n, q) / nn;
        double e[3];
        sub3(e, B, A);
        elen[i] = norm3(e);
    }
    const double nl = sqrt(nn);
    const double cs = fabs(denom) / (nl * norm3(ray->d));
    double rel = lam[0], clr = lam[0] * nl / elen[0];
    for (int i = 1; i < 3; ++i) {
        rel = fmin(rel, lam[i]);
        clr = fmin(clr, lam[i] * nl / elen[i]);
    }
    /* the ray passes the triangle where it spans along the ray, not at the
     * (possibly very distant) plane point of a grazing ray */
    const double dd = dot3(ray->d, ray->d);
    double tlo = OR_INF, thi = -OR_INF;
    for (int i = 0; i < 3; ++i) {
        double q0[3];
        sub3(q0, V[i], ray->o);
        const double tv = dot3(q0, ray->d) / dd;
        tlo = fmin(tlo, tv);
        thi = fmax(thi, tv);
    }
    c->rel = rel;
    c->clr = clr * cs;
    c->tref = fmin(fmax(t, tlo), thi);
    c->ok = rel >= 0.0;
    if (c->ok) {
        c->nroot = 1;
        c->t[0] = t;
        c->cs[0] = cs;
    }
}

static void eval_plane(const float* pl, const oray* ray, cand* c) {
    double n[3];
    load3f(n, pl);
    const double h = pl[3];
    const double nd = dot3(n, ray->d);
    c->valid = 0;
    c->ok = 0;
    c->nroot = 0;
    if (nd == 0.0) return;
    c->valid = 1;
    const double t = (h - dot3(n, ray->o)) / nd;
    const double cs = fabs(nd) / (norm3(n) * norm3(ray->d));
    c->rel = cs;
    c->clr = OR_INF;
    c->tref = t;
    c->ok = 1;
    c->nroot = 1;
    c->t[0] = t;
    c->cs[0] = cs;
}

static int64_t n_prims(const or_scene* sc) { return sc->n_spheres + sc->n_tris + sc->n_planes; }

/* Per-call scene view: the input arrays plus a bounding sphere per triangle
 * (centroid and the largest vertex distance).  The bounding spheres are a
 * per-primitive quantity, not an acceleration structure: every primitive is
 * still examined for every ray. */
typedef struct {
    const or_scene* in;
    double* tb;   /* [n_tris][4] cx cy cz R */
} oscene;

static int oscene_init(oscene* S, const or_scene* in) {
    S->in = in;
    S->tb = NULL;
    if (in->n_tris <= 0) return 0;
    S->tb = (double*)malloc(sizeof(double) * 4 * (size_t)in->n_tris);
    if (!S->tb) return -1;
    for (int64_t i = 0; i < in->n_tris; ++i) {
        const float* tv = in->tris + 9 * i;
        double c[3] = {0, 0, 0};
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j) c[j] += tv[3 * k + j] / 3.0;
        double R = 0.0;
        for (int k = 0; k < 3; ++k) {
            double q[3] = {tv[3 * k] - c[0], tv[3 * k + 1] - c[1], tv[3 * k + 2] - c[2]};
            R = fmax(R, norm3(q));
        }
        double* b = S->tb + 4 * i;
        b[0] = c[0]; b[1] = c[1]; b[2] = c[2]; b[3] = R;
    }
    return 0;
}

static void oscene_free(oscene* S) { free(S->tb); }

/* A triangle the ray passes far from is robustly missed: if the ray's line
 * misses the triangle's bounding sphere by more than twice max(cap * R,
 * 1e4 * cap * envelope), no admissible perturbation reaches it and its miss
 * margin exceeds the cap.  It is also skipped when its whole extent along the
 * ray lies outside the window [lo, hi] of parameters that can still matter. */
static int tri_skip(const oscene* S, int64_t j, const oray* ray, double lo, double hi) {
    const double* b = S->tb + 4 * j;
    double f[3] = {b[0] - ray->o[0], b[1] - ray->o[1], b[2] - ray->o[2]};
    const double dd = dot3(ray->d, ray->d);
    const double tc = dot3(f, ray->d) / dd;
    const double R = b[3];
    const double dl = sqrt(dd);
    if (tc + R / dl < lo || tc - R / dl > hi) return 1;
    double perp2 = dot3(f, f) - tc * tc * dd;
    if (perp2 < 0) perp2 = 0;
    const double gap = sqrt(perp2) - R;
    const double guard = 2.0 * fmax(MARGIN_CAP * R, 1e4 * MARGIN_CAP * envelope(ray, fabs(tc) + R / dl));
    return gap > guard;
}

/* ids: spheres 0..ns-1, then triangles, then planes.  [lo, hi] is the window
 * of ray parameters that can still matter to the query. */
static void eval_prim(const oscene* S, int64_t id, const oray* ray, double lo, double hi, cand* c) {
    const or_scene* sc = S->in;
    if (id < sc->n_spheres) {
        eval_sphere(sc->spheres + 4 * id, ray, c);
    } else if (id < sc->n_spheres + sc->n_tris) {
        const int64_t j = id - sc->n_spheres;
        if (tri_skip(S, j, ray, lo, hi)) {
            c->valid = 0;
            c->ok = 0;
            c->nroot = 0;
            return;
        }
        eval_tri(sc->tris + 9 * j, ray, c);
    } else {
        eval_plane(sc->planes + 4 * (id - sc->n_spheres - sc->n_tris), ray, c);
    }
}

/* margin contribution of a root t_c lying outside (0, tmax) or of the hit's own root */
static double range_margin(const oray* ray, double tc, double cs) {
    const double oscale = fmax(1.0, maxabs3(ray->o));
    double m = fabs(tc) / oscale;
    m = fmin(m, 1e-4 * fabs(tc) * fmax(cs, 1e-12) / (ray->so + EA * maxabs3(ray->o) + 1e-30));
    if (isfinite(ray->tmax)) {
        const double dt = fabs(ray->tmax - tc);
        m = fmin(m, dt / ray->tmax);
        m = fmin(m, 1e-4 * dt * fmax(cs, 1e-12) / envelope(ray, ray->tmax));
    }
    return m;
}

/* margin of a shape decision (inside when ok, outside otherwise) */
static double shape_margin(const oray* ray, const cand* c) {
    double m = fabs(c->rel);
    if (isfinite(c->clr)) m = fmin(m, 1e-4 * fabs(c->clr) / envelope(ray, c->tref));
    return m;
}

typedef struct {
    double t;
    int64_t id;
    double cs;
    double margin;
} hitrec;

/* Closest hit over every primitive (brute force), ties to the smaller id. */
static void closest_hit(const oscene* S, const oray* ray, hitrec* out) {
    const int64_t N = n_prims(S->in);
    double t1 = OR_INF, cs1 = 1.0, t2 = OR_INF, cs2 = 1.0;
    int64_t id1 = -1;
    cand best;
    memset(&best, 0, sizeof best);
    double m_other = MARGIN_CAP;   /* margins of primitives that are not the hit */
    const double oscale = fmax(1.0, maxabs3(ray->o));
    for (int64_t id = 0; id < N; ++id) {
        cand c;
        /* slack of the relevance window, against the running best */
        const double tb = fmin(t1, ray->tmax);
        const double slack = 1e-3 * fmax(oscale, isfinite(tb) ? tb : 0.0);
        eval_prim(S, id, ray, -slack, tb + slack, &c);
        if (!c.valid) continue;
        int hit_root = -1;
        if (c.ok) {
            for (int i = 0; i < c.nroot; ++i)
                if (c.t[i] > 0.0 && c.t[i] < ray->tmax) { hit_root = i; break; }
        }
        if (hit_root >= 0) {
            const double th = c.t[hit_root];
            if (th < t1 || (th == t1 && id < id1)) {
                /* previous best becomes a competitor */
                if (id1 >= 0 && t1 < t2) { t2 = t1; cs2 = cs1; }
                t1 = th; cs1 = c.cs[hit_root]; id1 = id; best = c;
            } else if (th < t2) {
                t2 = th; cs2 = c.cs[hit_root];
            }
            /* the primitive's other roots near the segment ends */
            for (int i = 0; i < c.nroot; ++i)
                if (i != hit_root && c.t[i] > -slack && c.t[i] < fmin(t1, ray->tmax) + slack)
                    m_other = fmin(m_other, range_margin(ray, c.t[i], c.cs[i]));
        } else if (c.ok) {
            /* shape passes but no root in (0, tmax): range decisions */
            for (int i = 0; i < c.nroot; ++i)
                if (c.t[i] > -slack && c.t[i] < tb + slack)
                    m_other = fmin(m_other, range_margin(ray, c.t[i], c.cs[i]));
        } else {
            /* shape test fails: relevant only if the shape decision lies within the window */
            if (c.tref > -slack && c.tref < tb + slack) m_other = fmin(m_other, shape_margin(ray, &c));
        }
    }
    out->t = t1;
    out->id = id1;
    out->cs = cs1;
    double m = m_other;
    if (id1 >= 0) {
        m = fmin(m, shape_margin(ray, &best));
        m = fmin(m, range_margin(ray, t1, cs1));
        if (isfinite(t2)) {
            const double gap = t2 - t1;
            m = fmin(m, gap / t1);
            m = fmin(m, 1e-4 * gap * fmin(cs1, cs2) / envelope(ray, t2));
        }
    }
    out->margin = fmin(m, MARGIN_CAP);
}

/* Any hit in (0, tmax): the shadow loop of Algorithm 1.  Returns 1 if blocked. */
static int any_hit(const oscene* S, const oray* ray, double* margin) {
    const int64_t N = n_prims(S->in);
    double best_blocker = -1.0;  /* best robustness among blockers */
    double m_free = MARGIN_CAP;  /* robustness of "nothing blocks" */
    const double slack = 1e-3 * fmax(fmax(1.0, maxabs3(ray->o)), ray->tmax);
    for (int64_t id = 0; id < N; ++id) {
        cand c;
        eval_prim(S, id, ray, -slack, ray->tmax + slack, &c);
        if (!c.valid) continue;
        if (c.ok) {
            for (int i = 0; i < c.nroot; ++i) {
                const double tc = c.t[i];
                if (tc > 0.0 && tc < ray->tmax) {
                    double mb = fmin(shape_margin(ray, &c), range_margin(ray, tc, c.cs[i]));
                    best_blocker = fmax(best_blocker, mb);
                } else if (tc > -slack && tc < ray->tmax + slack) {
                    m_free = fmin(m_free, range_margin(ray, tc, c.cs[i]));
                }
            }
        } else if (c.tref > -slack && c.tref < ray->tmax + slack) {
            m_free = fmin(m_free, shape_margin(ray, &c));
        }
        /* one clearly robust blocker settles the query (break on first blocker) */
        if (best_blocker >= 1e-2) break;
    }
    if (best_blocker >= 0.0) {
        *margin = fmin(best_blocker, MARGIN_CAP);
        return 1;
    }
    *margin = m_free;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* shading: Whitted recursion with Phong local illumination                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    const oscene* S;
    const or_scene* sc;
    const or_params* p;
    double margin;
    int32_t* counts;   /* [D+1][2]: closest-hit queries, shadow queries */
    double* rec;       /* optional ray log: [cap][RECW] */
    int64_t rec_n, rec_cap;
    double lloc;       /* bound on any surface's local radiance */
    double ignored;    /* worst-case RGB effect of decisions left out of the margin */
    int cache_depth;   /* < 0: off; else hits at this depth are recorded, not shaded */
    double* cache_rec; /* [cap][13]: list index, x[3], N_f[3], V[3], w[3] */
    int64_t* cache_n;  /* shared record counter */
    int64_t cache_cap;
    int64_t list_index;
    int32_t sample;    /* sample (pass) index: selects the area lights' sample points */
    int64_t pixel;     /* pixel index (row-major): with sample and depth, keys the path's random numbers */
    double gmax;       /* bound on the weight factor of one bounce (1 without global illumination) */
} pctx;

/* A decision whose worst-case effect on the sample's radiance is at most
 * RGB_IRRELEVANT (and while the sample's total of such effects stays within
 * RGB_BUDGET) cannot move the result by the 1e-3 RGB tolerance: it is left
 * out of the sample's margin. */
#define RGB_IRRELEVANT 1e-4
#define RGB_BUDGET 3e-4

static void note_margin(pctx* P, double m, double effect) {
    if (m > 1e-4) {
        P->margin = fmin(P->margin, m);
        return;
    }
    if (effect <= RGB_IRRELEVANT && P->ignored + effect <= RGB_BUDGET) {
        P->ignored += effect;
        return;
    }
    P->margin = fmin(P->margin, m);
}

/* bound on the radiance of a ray at depth k: local radiance at most lloc per
 * level, each level's weight factor at most gmax (1 for Whitted recursion:
 * k_r <= 1, F + (1 - F) = 1), plus the background */
static double radiance_bound(const pctx* P, int k) {
    const double* bg = P->p->bg;
    double b = 0.0, g = 1.0;
    for (int j = k; j <= P->p->max_depth; ++j) {
        b += g * P->lloc;
        g *= P->gmax;
    }
    return b + g / P->gmax * fmax(bg[0], fmax(bg[1], bg[2]));
}

/* bound on one bounce's weight factor with global illumination: the sum of
 * the branch weights of the material (see trace), at least 1 */
static double bounce_bound(const or_scene* sc, const or_params* p) {
    double g = 1.0;
    if (!p->gi) return g;
    for (int m = 0; m < sc->n_materials; ++m) {
        const float* M = sc->materials + 10 * m;
        const double am = fmax(M[0], fmax(M[1], M[2]));
        const double spec = ((int)M[9] == MAT_DIELECTRIC) ? 1.0 : fmax(0.0, (double)M[7]);
        g = fmax(g, fmax(0.0, (double)M[4]) * am + spec);
    }
    return g;
}

static double local_bound(const or_scene* sc) {
    double mat = 0.0, amb = 0.0, lsum = 0.0;
    for (int m = 0; m < sc->n_materials; ++m) {
        const float* M = sc->materials + 10 * m;
        const double am = fmax(M[0], fmax(M[1], M[2]));
        amb = fmax(amb, M[3] * am);
        mat = fmax(mat, M[4] * am + M[5]);
    }
    for (int l = 0; l < sc->n_lights; ++l) {
        const float* L = sc->lights + LW * l;
        lsum += fmax(L[3], fmax(L[4], L[5]));
    }
    return amb + lsum * mat;
}

/* ray log record: kind (0 camera, 1 reflected, 2 refracted, 3 shadow, 4 diffuse), depth,
 * o[3], d[3], tmax, t (closest hit) or blocked (shadow), id, margin */
#define RECW 12
static void log_ray(pctx* P, int kind, int depth, const oray* r, double t_or_occ, int64_t id, double margin) {
    if (!P->rec || P->rec_n >= P->rec_cap) { if (P->rec) P->rec_n++; return; }
    double* q = P->rec + RECW * P->rec_n++;
    q[0] = kind; q[1] = depth;
    for (int i = 0; i < 3; ++i) { q[2 + i] = r->o[i]; q[5 + i] = r->d[i]; }
    q[8] = r->tmax; q[9] = t_or_occ; q[10] = (double)id; q[11] = margin;
}

static const float* mat_of(const or_scene* sc, int64_t id) {
    int32_t m;
    if (id < sc->n_spheres) m = sc->sphere_mat[id];
    else if (id < sc->n_spheres + sc->n_tris) m = sc->tri_mat[id - sc->n_spheres];
    else m = sc->plane_mat[id - sc->n_spheres - sc->n_tris];
    return sc->materials + 10 * m;
}

/* Outward geometric normal at x; returns the normal's own uncertainty. */
static double geom_normal(const or_scene* sc, int64_t id, const double* x, double ex, double* n) {
    if (id < sc->n_spheres) {
        const float* s = sc->spheres + 4 * id;
        double c[3];
        load3f(c, s);
        sub3(n, x, c);
        normalize3(n);
        return ex / s[3] + EA;
    } else if (id < sc->n_spheres + sc->n_tris) {
        const float* tv = sc->tris + 9 * (id - sc->n_spheres);
        double v0[3], v1[3], v2[3], e1[3], e2[3];
        load3f(v0, tv);
        load3f(v1, tv + 3);
        load3f(v2, tv + 6);
        sub3(e1, v1, v0);
        sub3(e2, v2, v0);
        cross3(n, e1, e2);
        normalize3(n);
        return EA;
    } else {
        const float* pl = sc->planes + 4 * (id - sc->n_spheres - sc->n_tris);
        load3f(n, pl);
        normalize3(n);
        return EA;
    }
}

static void trace(pctx* P, const oray* ray, int kind, int k, const double* w, double* out, int64_t* primary_id);

/* Global illumination (Eq. 8, the hemisphere integral, Section II) by path
 * tracing: where Whitted recursion follows every specular branch, a path
 * follows one branch per bounce, chosen at random among
 *   diffuse  weight W_d = k_d * albedo (per channel): the Lambertian part,
 *            BRDF k_d * albedo / pi, sampled with the cosine-weighted density
 *            cos(theta) / pi, so that the estimator's factor is W_d;
 *   reflect  weight k_r (mirror), or F (dielectric);
 *   refract  weight 1 - F (dielectric, no total internal reflection);
 * with probability m_x / S, m_x the largest channel of branch x's weight and
 * S the sum of the m_x, and factor W_x * S / m_x: the expectation is the sum
 * of W_x times the branch's radiance, the full branching sum.  The branch is
 * the first (in the order above, among branches with m_x > 0) with
 * u S < m_1 + ... + m_x, else the last; u = or_path_rand(.., k, 0).
 * The diffuse direction is normalize(N_f + s), s uniform on the unit sphere
 * (z = 1 - 2 xi1, phi = 2 pi xi2; xi = or_path_rand(.., k, 1 and 2)): a point
 * uniform on the unit sphere that touches the surface at the hit point, seen
 * from the hit point, is cosine-distributed about N_f.  The light sources are
 * reached only by the shadow rays (they are not geometry), so nothing is
 * counted twice. */
static void gi_bounce(pctx* P, const oray* ray, int k, const double* w, const double* x, const double* xs,
                      const double* nf, double sn, double so2, double eps_s, int entering, const float* m,
                      double* out) {
    const or_params* p = P->p;
    const double alb[3] = {m[0], m[1], m[2]};
    const double kd = m[4], kr = m[7], ior = m[8];
    const int type = (int)m[9];
    const double cosi = -dot3(ray->d, nf);
    const double wmax = fmax(w[0], fmax(w[1], w[2]));
    /* the specular branches: directions and weights as in Whitted recursion */
    double F = 0.0, T = 0.0;
    oray rf, tr;
    for (int i = 0; i < 3; ++i) {
        rf.o[i] = xs[i];
        rf.d[i] = ray->d[i] + 2.0 * cosi * nf[i];
    }
    normalize3(rf.d);
    rf.tmax = OR_INF;
    rf.so = so2;
    rf.sd = ray->sd + 2.0 * sn + EA;
    if (type == MAT_DIELECTRIC) {
        const double eta = entering ? 1.0 / ior : ior;
        const double k2 = 1.0 - eta * eta * (1.0 - cosi * cosi);
        note_margin(P, 1e-4 * fabs(k2) / (2.0 * eta * eta * (ray->sd + sn) + EA), wmax * radiance_bound(P, k + 1));
        const double r0 = ((ior - 1.0) / (ior + 1.0)) * ((ior - 1.0) / (ior + 1.0));
        F = 1.0;
        if (k2 >= 0.0) {
            const double ck = sqrt(k2);
            const double cc = entering ? cosi : ck;
            const double om = 1.0 - cc;
            F = r0 + (1.0 - r0) * om * om * om * om * om;
            T = 1.0 - F;
            for (int i = 0; i < 3; ++i) {
                tr.o[i] = x[i] - eps_s * nf[i];
                tr.d[i] = eta * ray->d[i] + (eta * cosi - ck) * nf[i];
            }
            normalize3(tr.d);
            tr.tmax = OR_INF;
            tr.so = so2;
            tr.sd = (ray->sd + 2.0 * sn) * (1.0 + eta / fmax(ck, 1e-2)) + EA;
        }
    } else if (kr > 0.0) {
        F = kr;
    }
    const double md = kd > 0.0 ? kd * fmax(alb[0], fmax(alb[1], alb[2])) : 0.0;
    const double mx[3] = {md, F, T};
    const double S = md + F + T;
    if (!(S > 0.0)) return;
    const uint32_t pix = (uint32_t)P->pixel, smp = (uint32_t)P->sample;
    const double u = or_path_rand(p->seed, p->frame, pix, smp, (uint32_t)k, 0);
    int last = -1, pick = -1;
    double cum = 0.0, gap = OR_INF;
    for (int b = 0; b < 3; ++b) {
        if (!(mx[b] > 0.0)) continue;
        if (last >= 0) gap = fmin(gap, fabs(u * S - cum) / S);   /* the boundary between two branches */
        cum += mx[b];
        if (pick < 0 && u * S < cum) pick = b;
        last = b;
    }
    if (pick < 0) pick = last;
    double f[3];
    if (gap < OR_INF) note_margin(P, gap, wmax * S * radiance_bound(P, k + 1));
    if (pick == 0) {
        for (int i = 0; i < 3; ++i) f[i] = kd * alb[i] * S / md;
        const double xi1 = or_path_rand(p->seed, p->frame, pix, smp, (uint32_t)k, 1);
        const double xi2 = or_path_rand(p->seed, p->frame, pix, smp, (uint32_t)k, 2);
        const double z = 1.0 - 2.0 * xi1, r = sqrt(fmax(0.0, 1.0 - z * z)), phi = 2.0 * M_PI * xi2;
        const double sph[3] = {r * cos(phi), r * sin(phi), z};
        oray dr;
        for (int i = 0; i < 3; ++i) {
            dr.o[i] = xs[i];
            dr.d[i] = nf[i] + sph[i];
        }
        const double len = norm3(dr.d);
        /* the direction is ill-conditioned where s is nearly -N_f */
        note_margin(P, fmin(len, 1e-4 * len / (sn + 4.0 * EA)), wmax * S * radiance_bound(P, k + 1));
        if (!(len > 0.0)) return;
        for (int i = 0; i < 3; ++i) dr.d[i] /= len;
        dr.tmax = OR_INF;
        dr.so = so2;
        dr.sd = (sn + 4.0 * EA) / len + EA;
        double wc[3], lc[3];
        for (int i = 0; i < 3; ++i) wc[i] = w[i] * f[i];
        trace(P, &dr, 4, k + 1, wc, lc, NULL);
        for (int i = 0; i < 3; ++i) out[i] += f[i] * lc[i];
    } else {
        double wc[3], lc[3];
        for (int i = 0; i < 3; ++i) wc[i] = w[i] * S;
        trace(P, pick == 1 ? &rf : &tr, pick == 1 ? 1 : 2, k + 1, wc, lc, NULL);
        for (int i = 0; i < 3; ++i) out[i] += S * lc[i];
    }
}

/* w: the ray's throughput (its weight in the sample's radiance) */
static void trace(pctx* P, const oray* ray, int kind, int k, const double* w, double* out, int64_t* primary_id) {
    const or_scene* sc = P->sc;
    const or_params* p = P->p;
    const double wmax = fmax(w[0], fmax(w[1], w[2]));
    P->counts[2 * k + 0] += 1;
    hitrec h;
    closest_hit(P->S, ray, &h);
    note_margin(P, h.margin, wmax * radiance_bound(P, k));
    log_ray(P, kind, k, ray, h.t, h.id, h.margin);
    if (primary_id) *primary_id = h.id;
    if (h.id < 0) {
        out[0] = p->bg[0]; out[1] = p->bg[1]; out[2] = p->bg[2];
        return;
    }
    double x[3], ng[3], nf[3], v[3];
    for (int i = 0; i < 3; ++i) x[i] = ray->o[i] + h.t * ray->d[i];
    const double ex = envelope(ray, h.t);
    const double sn = geom_normal(sc, h.id, x, ex, ng);
    const double dn = dot3(ray->d, ng);
    const int entering = dn < 0.0;
    if (k == P->cache_depth) {
        /* learned form: the hit's radiance comes from the cache; record its query */
        const int64_t slot = __atomic_fetch_add(P->cache_n, 1, __ATOMIC_RELAXED);
        if (slot < P->cache_cap) {
            double* q = P->cache_rec + 13 * slot;
            q[0] = (double)P->list_index;
            for (int i = 0; i < 3; ++i) {
                q[1 + i] = x[i];
                q[4 + i] = entering ? ng[i] : -ng[i];
                q[7 + i] = -ray->d[i];
                q[10 + i] = w[i];
            }
        }
        out[0] = out[1] = out[2] = 0.0;
        return;
    }
    /* which side faces the ray is a discrete decision (two-sided shading) */
    note_margin(P, fmin(fabs(dn), 1e-4 * fabs(dn) / (ray->sd + sn + EA)), wmax * radiance_bound(P, k));
    for (int i = 0; i < 3; ++i) {
        nf[i] = entering ? ng[i] : -ng[i];
        v[i] = -ray->d[i];
    }
    const float* m = mat_of(sc, h.id);
    const double alb[3] = {m[0], m[1], m[2]};
    const double ka = m[3], kd = m[4], ks = m[5], shin = m[6], kr = m[7], ior = m[8];
    const int type = (int)m[9];
    const double eps_s = p->eps * fmax(1.0, maxabs3(x));
    const double so2 = ex + EA * maxabs3(x);
    double xs[3];
    for (int i = 0; i < 3; ++i) xs[i] = x[i] + eps_s * nf[i];

    /* ambient: white ambient light of unit intensity */
    double local[3];
    for (int i = 0; i < 3; ++i) local[i] = ka * alb[i];
    for (int l = 0; l < sc->n_lights; ++l) {
        const float* L = sc->lights + LW * l;
        double lp[3], lv[3];
        or_light_point(L, p->seed, p->frame, P->sample, l, lp);
        sub3(lv, lp, x);
        normalize3(lv);
        const double ndl = dot3(nf, lv);
        if (ndl <= 0.0) continue;
        double rr[3];
        for (int i = 0; i < 3; ++i) rr[i] = 2.0 * ndl * nf[i] - lv[i];   /* Phong mirror direction of L */
        const double rv = fmax(0.0, dot3(rr, v));
        const double spec = ks * pow(rv, shin);
        double c[3];
        double cmax = 0.0;
        for (int i = 0; i < 3; ++i) {
            c[i] = (double)L[3 + i] * (kd * alb[i] * ndl + spec);
            cmax = fmax(cmax, c[i]);
        }
        if (!(cmax > 0.0)) continue;
        oray sr;
        double sdir[3];
        sub3(sdir, lp, xs);
        const double dist = norm3(sdir);
        for (int i = 0; i < 3; ++i) { sr.o[i] = xs[i]; sr.d[i] = sdir[i] / dist; }
        sr.tmax = dist;
        sr.so = so2;
        sr.sd = so2 / dist + EA;
        P->counts[2 * k + 1] += 1;
        double sm;
        const int blocked = any_hit(P->S, &sr, &sm);
        note_margin(P, sm, fmax(w[0] * c[0], fmax(w[1] * c[1], w[2] * c[2])));
        log_ray(P, 3, k, &sr, (double)blocked, -1, sm);
        if (!blocked)
            for (int i = 0; i < 3; ++i) local[i] += c[i];
    }
    for (int i = 0; i < 3; ++i) out[i] = local[i];
    if (k >= p->max_depth) return;
    if (p->gi) {
        gi_bounce(P, ray, k, w, x, xs, nf, sn, so2, eps_s, entering, m, out);
        return;
    }

    const double cosi = -dot3(ray->d, nf);   /* > 0 */
    oray rf;
    for (int i = 0; i < 3; ++i) {
        rf.o[i] = xs[i];
        rf.d[i] = ray->d[i] + 2.0 * cosi * nf[i];
    }
    normalize3(rf.d);
    rf.tmax = OR_INF;
    rf.so = so2;
    rf.sd = ray->sd + 2.0 * sn + EA;

    if (type == MAT_DIELECTRIC) {
        const double eta = entering ? 1.0 / ior : ior;
        const double k2 = 1.0 - eta * eta * (1.0 - cosi * cosi);
        note_margin(P, 1e-4 * fabs(k2) / (2.0 * eta * eta * (ray->sd + sn) + EA), wmax * radiance_bound(P, k + 1));
        const double r0 = ((ior - 1.0) / (ior + 1.0)) * ((ior - 1.0) / (ior + 1.0));
        double F = 1.0;
        oray tr;
        int has_t = 0;
        if (k2 >= 0.0) {
            const double ck = sqrt(k2);
            const double cc = entering ? cosi : ck;
            const double om = 1.0 - cc;
            F = r0 + (1.0 - r0) * om * om * om * om * om;
            for (int i = 0; i < 3; ++i) {
                tr.o[i] = x[i] - eps_s * nf[i];
                tr.d[i] = eta * ray->d[i] + (eta * cosi - ck) * nf[i];
            }
            normalize3(tr.d);
            tr.tmax = OR_INF;
            tr.so = so2;
            tr.sd = (ray->sd + 2.0 * sn) * (1.0 + eta / fmax(ck, 1e-2)) + EA;
            has_t = 1;
        }
        double lr[3], wr[3] = {w[0] * F, w[1] * F, w[2] * F};
        trace(P, &rf, 1, k + 1, wr, lr, NULL);
        for (int i = 0; i < 3; ++i) out[i] += F * lr[i];
        if (has_t) {
            double lt[3], wt[3] = {w[0] * (1.0 - F), w[1] * (1.0 - F), w[2] * (1.0 - F)};
            trace(P, &tr, 2, k + 1, wt, lt, NULL);
            for (int i = 0; i < 3; ++i) out[i] += (1.0 - F) * lt[i];
        }
    } else if (kr > 0.0) {
        double lr[3], wr[3] = {w[0] * kr, w[1] * kr, w[2] * kr};
        trace(P, &rf, 1, k + 1, wr, lr, NULL);
        for (int i = 0; i < 3; ++i) out[i] += kr * lr[i];
    }
}

/* ------------------------------------------------------------------------ */
/* threading                                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int64_t next;
    pthread_mutex_t mu;
    void (*fn)(void* ctx, int64_t i);
    void* ctx;
} pool;

static void* pool_worker(void* arg) {
    pool* P = (pool*)arg;
    for (;;) {
        pthread_mutex_lock(&P->mu);
        int64_t i = P->next++;
        pthread_mutex_unlock(&P->mu);
        if (i >= P->n) break;
        P->fn(P->ctx, i);
    }
    return NULL;
}

static void run_parallel(int64_t n, int nthreads, void (*fn)(void*, int64_t), void* ctx) {
    if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > n) nthreads = (int)(n > 0 ? n : 1);
    pool P = {n, 0, PTHREAD_MUTEX_INITIALIZER, fn, ctx};
    pthread_t th[256];
    for (int i = 0; i < nthreads; ++i) pthread_create(&th[i], NULL, pool_worker, &P);
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
}

/* ------------------------------------------------------------------------ */
/* exported entry points                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    const oscene* S;
    const or_scene* sc;
    const or_camera* cam;
    const or_params* p;
    const int64_t* pixels;
    double* rgb;
    int64_t* ids;
    double* margin;
    int32_t* counts;
    double* rgb_s;      /* [n][spp][3] per-sample radiance, or NULL */
    double* margin_s;   /* [n][spp] per-sample margin, or NULL */
    int cache_depth;
    double* cache_rec;
    int64_t* cache_n;
    int64_t cache_cap;
} render_job;

static void render_one(void* vctx, int64_t i) {
    render_job* J = (render_job*)vctx;
    const int D = J->p->max_depth;
    int32_t local_counts[2 * 64];
    memset(local_counts, 0, sizeof local_counts);
    pctx P = {J->S, J->sc, J->p, MARGIN_CAP, local_counts, NULL, 0, 0, local_bound(J->sc), 0.0,
              J->cache_depth, J->cache_rec, J->cache_n, J->cache_cap, i, 0, J->pixels[i], bounce_bound(J->sc, J->p)};
    const double one[3] = {1.0, 1.0, 1.0};
    double acc[3] = {0, 0, 0};
    const int64_t pix = J->pixels[i];
    for (int s = 0; s < J->p->spp; ++s) {
        oray r;
        or_camera_ray(J->cam, J->p, pix, s, r.o, r.d);
        r.tmax = OR_INF;
        r.so = EA * maxabs3(r.o);
        r.sd = EA;
        double L[3];
        int64_t pid = -1;
        const double m_before = P.margin;
        P.margin = MARGIN_CAP;
        P.ignored = 0.0;
        P.sample = s;
        trace(&P, &r, 0, 0, one, L, &pid);
        for (int c = 0; c < 3; ++c) acc[c] += L[c];
        if (J->ids) J->ids[i * J->p->spp + s] = pid;
        if (J->rgb_s)
            for (int c = 0; c < 3; ++c) J->rgb_s[(i * J->p->spp + s) * 3 + c] = L[c];
        if (J->margin_s) J->margin_s[i * J->p->spp + s] = P.margin;
        P.margin = fmin(P.margin, m_before);
    }
    for (int c = 0; c < 3; ++c) J->rgb[3 * i + c] = acc[c] / J->p->spp;
    if (J->margin) J->margin[i] = P.margin;
    if (J->counts) memcpy(J->counts + i * 2 * (D + 1), local_counts, sizeof(int32_t) * 2 * (D + 1));
}

/* Render a list of pixels.  rgb [n][3], ids [n][spp] (or NULL), margin [n]
 * (min over the pixel's ray trees, or NULL), counts [n][D+1][2] (or NULL),
 * rgb_s [n][spp][3] and margin_s [n][spp] per sample (or NULL). */
int or_render(const or_scene* sc, const or_camera* cam, const or_params* p, const int64_t* pixels, int64_t n,
              int32_t nthreads, double* rgb, int64_t* ids, double* margin, int32_t* counts, double* rgb_s,
              double* margin_s) {
    if (p->max_depth < 0 || p->max_depth > 63 || p->spp < 1) return -1;
    oscene S;
    if (oscene_init(&S, sc) != 0) return -2;
    render_job J = {&S, sc, cam, p, pixels, rgb, ids, margin, counts, rgb_s, margin_s, -1, NULL, NULL, 0};
    run_parallel(n, nthreads, render_one, &J);
    oscene_free(&S);
    return 0;
}

typedef struct {
    const oscene* S;
    const double* rays;
    double* t;
    int64_t* id;
    uint8_t* occ;
    double* margin;
    double* uv;
} ray_job;

/* Surface coordinates of a hit at ray parameter t on primitive id:
 *   triangle: the barycentric weights (u, v) of its second and third vertex,
 *     so that the hit point is (1-u-v) v0 + u v1 + v v2, from the edge
 *     functions at the plane point (the same construction as eval_tri);
 *   sphere: the unit outward normal n = (x - c)/r in spherical coordinates,
 *     u = (atan2(n_z, n_x) + pi) / (2 pi) (longitude), v = acos(n_y) / pi
 *     (polar angle from +y), both in [0, 1];
 *   plane: (0, 0) (a plane carries no parameterisation). */
static void hit_uv(const or_scene* sc, const oray* ray, int64_t id, double t, double* uv) {
    uv[0] = uv[1] = 0.0;
    if (id < 0) return;
    double p[3];
    for (int k = 0; k < 3; ++k) p[k] = ray->o[k] + t * ray->d[k];
    if (id < sc->n_spheres) {
        const float* s = sc->spheres + 4 * id;
        double n[3];
        for (int k = 0; k < 3; ++k) n[k] = (p[k] - (double)s[k]) / (double)s[3];
        const double ny = fmax(-1.0, fmin(1.0, n[1]));
        uv[0] = (atan2(n[2], n[0]) + M_PI) / (2.0 * M_PI);
        uv[1] = acos(ny) / M_PI;
    } else if (id < sc->n_spheres + sc->n_tris) {
        const float* tv = sc->tris + 9 * (id - sc->n_spheres);
        double v0[3], v1[3], v2[3], e1[3], e2[3], n[3], a[3], b[3], q[3];
        load3f(v0, tv);
        load3f(v1, tv + 3);
        load3f(v2, tv + 6);
        sub3(e1, v1, v0);
        sub3(e2, v2, v0);
        cross3(n, e1, e2);
        const double nn = dot3(n, n);
        /* weight of v1: the edge v2 -> v0 seen from p; weight of v2: the edge v0 -> v1 */
        sub3(a, v2, p);
        sub3(b, v0, p);
        cross3(q, a, b);
        uv[0] = dot3(n, q) / nn;
        sub3(a, v0, p);
        sub3(b, v1, p);
        cross3(q, a, b);
        uv[1] = dot3(n, q) / nn;
    }
}

static void load_ray(const double* R, oray* r) {
    for (int i = 0; i < 3; ++i) { r->o[i] = R[i]; r->d[i] = R[3 + i]; }
    r->tmax = R[6] > 0 ? R[6] : OR_INF;
    r->so = R[7];
    r->sd = R[8];
}

static void closest_one(void* vctx, int64_t i) {
    ray_job* J = (ray_job*)vctx;
    oray r;
    load_ray(J->rays + 9 * i, &r);
    hitrec h;
    closest_hit(J->S, &r, &h);
    J->t[i] = h.t;
    J->id[i] = h.id;
    J->margin[i] = h.margin;
    if (J->uv) hit_uv(J->S->in, &r, h.id, h.t, J->uv + 2 * i);
}

static void occluded_one(void* vctx, int64_t i) {
    ray_job* J = (ray_job*)vctx;
    oray r;
    load_ray(J->rays + 9 * i, &r);
    double m;
    J->occ[i] = (uint8_t)any_hit(J->S, &r, &m);
    J->margin[i] = m;
}

/* rays [n][9]: o(3), d(3), tmax (<= 0 means infinite), so, sd; uv [n][2]
 * (or NULL) receives the hit's surface coordinates (see hit_uv) */
int or_closest(const or_scene* sc, const double* rays, int64_t n, int32_t nthreads, double* t, int64_t* id,
               double* margin, double* uv) {
    oscene S;
    if (oscene_init(&S, sc) != 0) return -2;
    ray_job J = {&S, rays, t, id, NULL, margin, uv};
    run_parallel(n, nthreads, closest_one, &J);
    oscene_free(&S);
    return 0;
}

int or_occluded(const or_scene* sc, const double* rays, int64_t n, int32_t nthreads, uint8_t* occ,
                double* margin) {
    oscene S;
    if (oscene_init(&S, sc) != 0) return -2;
    ray_job J = {&S, rays, NULL, NULL, occ, margin, NULL};
    run_parallel(n, nthreads, occluded_one, &J);
    oscene_free(&S);
    return 0;
}

/* Ray tree of one pixel sample: every ray the recursion traces, in order.
 * rec [cap][12] (see log_ray); returns the number of rays (may exceed cap,
 * in which case only cap were written), or < 0 on error.  rgb [3] receives
 * the sample's radiance. */
int64_t or_ray_tree(const or_scene* sc, const or_camera* cam, const or_params* p, int64_t pixel, int32_t sample,
                    double* rec, int64_t cap, double* rgb) {
    if (p->max_depth < 0 || p->max_depth > 63) return -1;
    oscene S;
    if (oscene_init(&S, sc) != 0) return -2;
    int32_t counts[2 * 64];
    memset(counts, 0, sizeof counts);
    pctx P = {&S, sc, p, MARGIN_CAP, counts, rec, 0, cap, local_bound(sc), 0.0, -1, NULL, NULL, 0, 0, 0, pixel,
              bounce_bound(sc, p)};
    const double one[3] = {1.0, 1.0, 1.0};
    oray r;
    or_camera_ray(cam, p, pixel, sample, r.o, r.d);
    r.tmax = OR_INF;
    r.so = EA * maxabs3(r.o);
    r.sd = EA;
    int64_t pid;
    P.sample = sample;
    trace(&P, &r, 0, 0, one, rgb, &pid);
    oscene_free(&S);
    return P.rec_n;
}

/* Learned form: trace pixels with the recursion cut at cache_depth.  Hits at
 * that depth add nothing; each is recorded as (list index, x, N_f, V,
 * throughput w) in rec [cap][13] so that the caller adds w * max(cache(x, N_f,
 * V), 0).  Misses at that depth still return the background.  rgb [n][3] is
 * the radiance without the cache terms, margin [n] as or_render.  Returns the
 * number of records (may exceed cap; only cap are written). */
int64_t or_render_cache(const or_scene* sc, const or_camera* cam, const or_params* p, const int64_t* pixels,
                        int64_t n, int32_t cache_depth, int32_t nthreads, double* rgb, double* margin, double* rec,
                        int64_t cap) {
    if (p->max_depth < 0 || p->max_depth > 63 || p->spp < 1 || cache_depth < 0) return -1;
    oscene S;
    if (oscene_init(&S, sc) != 0) return -2;
    int64_t count = 0;
    render_job J = {&S, sc, cam, p, pixels, rgb, NULL, margin, NULL, NULL, NULL, cache_depth, rec, &count, cap};
    run_parallel(n, nthreads, render_one, &J);
    oscene_free(&S);
    return count;
}

typedef struct {
    const oscene* S;
    const or_params* p;
    const double* rays;
    int start_depth;
    double* L;
    double* margin;
    int32_t sample;
    const int64_t* pixels;   /* pixel of each ray (keys its path's random numbers), or NULL: the ray's index */
} radiance_job;

static void radiance_one(void* vctx, int64_t i) {
    radiance_job* J = (radiance_job*)vctx;
    int32_t counts[2 * 64];
    memset(counts, 0, sizeof counts);
    pctx P = {J->S, J->S->in, J->p, MARGIN_CAP, counts, NULL, 0, 0, local_bound(J->S->in), 0.0, -1, NULL, NULL, 0, 0,
              0, J->pixels ? J->pixels[i] : i, bounce_bound(J->S->in, J->p)};
    oray r;
    load_ray(J->rays + 9 * i, &r);
    const double one[3] = {1.0, 1.0, 1.0};
    P.sample = J->sample;
    trace(&P, &r, 0, J->start_depth, one, J->L + 3 * i, NULL);
    J->margin[i] = P.margin;
}

/* Radiance L(ray) of n rays that start at recursion depth start_depth (so
 * secondary rays spawn while depth < max_depth): the training targets of the
 * learned form.  rays [n][9] as or_closest; L [n][3]; margin [n].  With global
 * illumination the path of ray i draws its random numbers with the pixel key
 * pixels[i] (NULL: i) and the given sample. */
int or_radiance(const or_scene* sc, const or_params* p, const double* rays, int64_t n, int32_t start_depth,
                int32_t sample, int32_t nthreads, double* L, double* margin, const int64_t* pixels) {
    if (p->max_depth < 0 || p->max_depth > 63 || start_depth < 0 || start_depth > p->max_depth) return -1;
    oscene S;
    if (oscene_init(&S, sc) != 0) return -2;
    radiance_job J = {&S, p, rays, start_depth, L, margin, sample, pixels};
    run_parallel(n, nthreads, radiance_one, &J);
    oscene_free(&S);
    return 0;
}
