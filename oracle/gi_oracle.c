/*
 * FP64 CPU oracle for the per-pixel hot path of DDGI resampling
 * (Majercik, Mueller, Keller, Nowrouzezahrai, McGuire: "Dynamic Diffuse
 * Global Illumination Resampling", EGSR 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP implementation; the only
 * thing both sides see is the seeded input arrays (scene, camera, probe grid)
 * and the published Philox4x32-10 definition, which each side implements on
 * its own.
 *
 * Style: plain, single-threaded, double precision, no blocking or fusion.
 * Every pass is written per pixel in the order of the method so that it can
 * be checked against the paper by eye.  Pixels can be evaluated one by one
 * (pixel lists) so that full-size frames can be checked on samples.
 *
 * Record layouts (all double):
 *   G-buffer pixel  [14]: pos[3] nrm[3] albedo[3] emit[3] view_depth prim
 *   reservoir       [14]: y[3] n_y[3] L[3] wsum W M tag prim
 *   probe textures : irr[P][(Ni+2)^2][3] (E/pi), dep[P][(Nd+2)^2][2] (mean, mean^2);
 *                    texels are kept at their storage precision: with
 *                    o_probes.texel = 0 at full precision, with texel = 1
 *                    as binary16 (o_round_half) irradiance, and for depth a
 *                    binary16 mean and variance with the mean square rebuilt
 *                    from them (dep_texel); the update stores them so, the
 *                    query reads a caller's tile so
 * A reservoir whose sample left the scene stores the direction in y and a
 * zero normal in n_y.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

/* Optional OpenMP pixel loops (build with -fopenmp): every pixel or probe
 * iteration reads shared inputs and writes only its own outputs, so the
 * results are bitwise identical for any thread count.  One thread unless
 * o_set_threads says otherwise. */
static int o_threads = 1;
void o_set_threads(int n) { o_threads = n < 1 ? 1 : n; }
int o_openmp(void)
{
#ifdef _OPENMP
    return 1;
#else
    return 0;
#endif
}
#define O_PARALLEL _Pragma("omp parallel for schedule(dynamic, 16) num_threads(o_threads) if(o_threads > 1)")

#define O_MISS 0xFFFFFFFFu
#define O_PI 3.14159265358979323846
#define O_INF (1.0 / 0.0)

/* ---------------------------------------------------------------------------
 * Inputs
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t n_prims;
    int32_t has_room;
    const double *prims;            /* n_prims x 16 records (see scene generator) */
    double room_lo[3], room_hi[3];
    double wall_albedo[3], wall_emit[3];
    double sky[3];
    double eps;                     /* ray-origin offset along the surface normal */
    int32_t glossy;                 /* 1: primitives carry a specular layer (record slots 11, 15) */
    int32_t pad;
} o_scene;

typedef struct {
    double eye[3], fwd[3], right[3], up[3];
    double tan_half_fovy;
    int32_t width, height;
} o_camera;

typedef struct {
    int32_t dims[3];
    int32_t irr_res, dep_res;
    double lo[3], spacing[3];
    double bias_dist;               /* view-path bias distance d */
    double var_floor;               /* Chebyshev variance floor */
    double d_max;                   /* depth clamp for probe rays */
    const double *irr;
    const double *dep;
    /* learned cache used as the target instead of the probe query (NULL: probes) */
    const double *mlp;              /* 17731 parameters, layout of oracle/mlp_ref.py */
    int32_t mlp_prec;               /* 0: FP64, 1: BF16 operands */
    int32_t texel;                  /* texel storage: 0 full precision, 1 binary16 */
    double mlp_lo[3], mlp_hi[3];    /* position normalisation box */
} o_probes;

typedef struct {
    int32_t M;                      /* candidates per pixel */
    int32_t k;                      /* spatial neighbours */
    int32_t unbiased;               /* 1: 1/Z with visibility; 0: 1/M */
    int32_t M_light;                /* emitter-sampled candidates per pixel */
    double radius;                  /* spatial radius in pixels */
    double g_max;                   /* geometry-term bound */
    double cos_n;                   /* reuse normal threshold */
    double depth_rel;               /* reuse relative depth threshold */
    double m_cap;                   /* temporal history cap (multiple of the per-frame candidate count) */
    int32_t subsample;              /* n: pixel (x, y) draws candidates in frame f iff (x+y+f) % n == 0 */
    int32_t pad;
    double eye[3];                  /* camera position of the current frame (glossy primary vertices) */
    double eye_prev[3];             /* camera position of the previous frame (temporal history) */
    double foot_c;                  /* footprint threshold c of the shading recursion (Eq. 8) */
    int32_t glossy_depth;           /* most glossy vertices the shading recursion visits */
    int32_t pad2;
} o_params;

enum { GB_POS = 0, GB_NRM = 3, GB_ALB = 6, GB_EMIT = 9, GB_DEPTH = 12, GB_PRIM = 13, GB_N = 14 };
enum { R_Y = 0, R_NY = 3, R_L = 6, R_WSUM = 9, R_W = 10, R_M = 11, R_TAG = 12, R_PRIM = 13, R_N = 14 };

/* ---------------------------------------------------------------------------
 * Small vector helpers
 * ------------------------------------------------------------------------- */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double lum(const double *c) { return 0.2126 * c[0] + 0.7152 * c[1] + 0.0722 * c[2]; }
static void normalize3(double *v)
{
    double l = sqrt(dot3(v, v));
    v[0] /= l; v[1] /= l; v[2] /= l;
}
static double sgn(double v) { return v >= 0.0 ? 1.0 : -1.0; }

/* ---------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
 * multiplications whose high and low halves are crossed and xored with the
 * key; the key advances by the Weyl constants between rounds.
 * Counter layout of this method: (pixel or probe, frame, pass, block);
 * key = (seed low word, seed high word).
 * ------------------------------------------------------------------------- */
void o_philox(uint32_t k0, uint32_t k1, const uint32_t *ctr, uint32_t *out)
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* uniform in [0,1) from the top 24 bits: exactly representable in f32 and f64 */
static double u01(uint32_t v) { return (double)(v >> 8) * (1.0 / 16777216.0); }

static void rand4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, double *u)
{
    uint32_t ctr[4] = {c0, c1, c2, c3}, out[4];
    o_philox((uint32_t)seed, (uint32_t)(seed >> 32), ctr, out);
    for (int i = 0; i < 4; ++i) u[i] = u01(out[i]);
}

enum { PASS_INITIAL = 0, PASS_TEMPORAL = 1, PASS_SPATIAL0 = 2, PASS_PROBE = 9,
       PASS_GLOSSY_CAND = 14, PASS_GLOSSY_PROBE = 15, PASS_GLOSSY_SHADE = 16 };

/* ---------------------------------------------------------------------------
 * Sampling
 * ------------------------------------------------------------------------- */
/* Cosine-weighted direction about n (the Lambertian BSDF sampling of step 1,
 * Sec. 3.1): disk point (sqrt(u1) cos 2pi u0, sqrt(u1) sin 2pi u0), lifted to
 * the hemisphere, expressed in the orthonormal basis of Duff et al. 2017. */
static void onb(const double *n, double *t, double *bt)
{
    double s = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (s + n[2]);
    double b = n[0] * n[1] * a;
    t[0] = 1.0 + s * n[0] * n[0] * a; t[1] = s * b; t[2] = -s * n[0];
    bt[0] = b; bt[1] = s + n[1] * n[1] * a; bt[2] = -n[1];
}

void o_cosine_dir(const double *n, double u0, double u1, double *w)
{
    double phi = 2.0 * O_PI * u0, r = sqrt(u1);
    double lx = r * cos(phi), ly = r * sin(phi), lz = sqrt(fmax(0.0, 1.0 - u1));
    double t[3], bt[3];
    onb(n, t, bt);
    for (int i = 0; i < 3; ++i) w[i] = lx * t[i] + ly * bt[i] + lz * n[i];
}

/* ---------------------------------------------------------------------------
 * Glossy layer (Sec. 3.3: the glossy transport T_fg, "in our case microfacet
 * models"): an isotropic GGX (Trowbridge-Reitz) lobe with separable Smith
 * masking and a constant grey specular weight k_s (no Fresnel term):
 *   f_g(wo, wi) = k_s D(h) G1(wo) G1(wi) / (4 (n.wo) (n.wi)),  h = (wo+wi)/|wo+wi|,
 *   D(h) = a^2 / (pi ((n.h)^2 (a^2 - 1) + 1)^2),
 *   G1(v) = 2 (n.v) / ((n.v) + sqrt(a^2 + (1 - a^2) (n.v)^2)).
 * Sampling draws h with density D(h)(n.h) (Walter et al. 2007):
 * cos^2(theta_h) = (1 - u0) / (1 + (a^2 - 1) u0), phi = 2 pi u1, and reflects
 * wo about h; the solid-angle density of wi is D(h)(n.h) / (4 |wo.h|).
 * ------------------------------------------------------------------------- */
static double ggx_D(double nh, double a)
{
    double a2 = a * a, t = nh * nh * (a2 - 1.0) + 1.0;
    return a2 / (O_PI * t * t);
}

static double smith_G1(double nv, double a)
{
    double a2 = a * a;
    return 2.0 * nv / (nv + sqrt(a2 + (1.0 - a2) * nv * nv));
}

/* f_g / k_s; 0 unless both directions lie above the surface */
static double ggx_eval(const double *n, const double *wo, const double *wi, double a)
{
    double no = dot3(n, wo), ni = dot3(n, wi);
    if (no <= 0.0 || ni <= 0.0) return 0.0;
    double h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
    normalize3(h);
    return ggx_D(dot3(n, h), a) * smith_G1(no, a) * smith_G1(ni, a) / (4.0 * no * ni);
}

/* solid-angle density of sampling wi from the lobe about wo */
static double ggx_pdf(const double *n, const double *wo, const double *wi, double a)
{
    if (dot3(n, wi) <= 0.0 || dot3(n, wo) <= 0.0) return 0.0;
    double h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
    normalize3(h);
    double nh = dot3(n, h), oh = fabs(dot3(wo, h));
    return oh > 0.0 ? ggx_D(nh, a) * nh / (4.0 * oh) : 0.0;
}

/* a direction from the lobe about wo; returns 0 (and no direction) when the
 * reflected direction falls below the surface */
static int ggx_sample(const double *n, const double *wo, double a, double u0, double u1, double *wi)
{
    double c2 = (1.0 - u0) / (1.0 + (a * a - 1.0) * u0);
    double ct = sqrt(c2), st = sqrt(fmax(0.0, 1.0 - c2)), phi = 2.0 * O_PI * u1;
    double t[3], bt[3], h[3];
    onb(n, t, bt);
    for (int i = 0; i < 3; ++i) h[i] = st * cos(phi) * t[i] + st * sin(phi) * bt[i] + ct * n[i];
    double oh = dot3(wo, h);
    for (int i = 0; i < 3; ++i) wi[i] = 2.0 * oh * h[i] - wo[i];
    return dot3(n, wi) > 0.0 && dot3(n, wo) > 0.0;
}

void o_ggx(const double *n, const double *wo, const double *wi, double a, double *out)
{
    out[0] = ggx_eval(n, wo, wi, a);
    out[1] = ggx_pdf(n, wo, wi, a);
}

int o_ggx_sample(const double *n, const double *wo, double a, double u0, double u1, double *wi)
{
    return ggx_sample(n, wo, a, u0, u1, wi);
}

/* f_g / k_s and the sampling density for k directions wi (rows of 3) */
void o_ggx_many(const double *n, const double *wo, const double *wi, int64_t k, double a, double *f, double *pdf)
{
    for (int64_t i = 0; i < k; ++i) {
        f[i] = ggx_eval(n, wo, wi + 3 * i, a);
        pdf[i] = ggx_pdf(n, wo, wi + 3 * i, a);
    }
}

/* Uniform direction on the unit sphere (probe-update rays). */
void o_sphere_dir(double u0, double u1, double *w)
{
    double z = 1.0 - 2.0 * u0, phi = 2.0 * O_PI * u1;
    double r = sqrt(fmax(0.0, 1.0 - z * z));
    w[0] = r * cos(phi); w[1] = r * sin(phi); w[2] = z;
}

/* ---------------------------------------------------------------------------
 * Ray casting against the analytic scene (brute force, index order).
 * Hit rule: smallest t > 0 (and < tmax); equal t goes to the lower index;
 * the room walls follow the primitives with indices n + 2*axis + (hi side).
 * Normals are geometric and turned to face the incoming ray.
 * ------------------------------------------------------------------------- */
typedef struct { double t; uint32_t prim; double n[3]; } o_hit;

static int hit_sphere(const double *rec, const double *o, const double *d, double *t, double *n)
{
    double oc[3] = {o[0] - rec[0], o[1] - rec[1], o[2] - rec[2]};
    double r = rec[4];
    double b = dot3(oc, d);
    double c = dot3(oc, oc) - r * r;
    double disc = b * b - c;
    if (disc < 0.0) return 0;
    double s = sqrt(disc);
    double t0 = -b - s, t1 = -b + s, th;
    if (t0 > 0.0) th = t0;
    else if (t1 > 0.0) th = t1;
    else return 0;
    *t = th;
    for (int i = 0; i < 3; ++i) n[i] = (o[i] + th * d[i] - rec[i]) / r;
    if (dot3(n, d) > 0.0) for (int i = 0; i < 3; ++i) n[i] = -n[i];
    return 1;
}

static int hit_box(const double *rec, const double *o, const double *d, double *t, double *n)
{
    double tn = -O_INF, tf = O_INF;
    int an = 0, af = 0;
    for (int a = 0; a < 3; ++a) {
        double inv = 1.0 / d[a];
        double t1 = (rec[a] - rec[4 + a] - o[a]) * inv;
        double t2 = (rec[a] + rec[4 + a] - o[a]) * inv;
        double lo = fmin(t1, t2), hi = fmax(t1, t2);
        if (lo > tn) { tn = lo; an = a; }
        if (hi < tf) { tf = hi; af = a; }
    }
    if (tn > tf) return 0;
    int axis;
    if (tn > 0.0) { *t = tn; axis = an; }
    else if (tf > 0.0) { *t = tf; axis = af; }
    else return 0;
    n[0] = n[1] = n[2] = 0.0;
    n[axis] = -sgn(d[axis]);
    return 1;
}

static int hit_room(const o_scene *sc, const double *o, const double *d, double *t, double *n, uint32_t *wall)
{
    double best = O_INF;
    int ba = -1;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) continue;
        double ta = ((d[a] > 0.0 ? sc->room_hi[a] : sc->room_lo[a]) - o[a]) / d[a];
        if (ta > 0.0 && ta < best) { best = ta; ba = a; }
    }
    if (ba < 0) return 0;
    *t = best;
    n[0] = n[1] = n[2] = 0.0;
    n[ba] = -sgn(d[ba]);
    *wall = (uint32_t)sc->n_prims + 2u * (uint32_t)ba + (d[ba] > 0.0 ? 1u : 0u);
    return 1;
}

static int closest_hit(const o_scene *sc, const double *o, const double *d, double tmax, o_hit *h)
{
    h->t = tmax;
    h->prim = O_MISS;
    for (int i = 0; i < sc->n_prims; ++i) {
        const double *rec = sc->prims + 16 * i;
        uint32_t type = (uint32_t)rec[3];      /* 0 sphere, 1 box */
        double t, n[3];
        int ok = type == 0 ? hit_sphere(rec, o, d, &t, n) : hit_box(rec, o, d, &t, n);
        if (ok && t < h->t) {
            h->t = t; h->prim = (uint32_t)i;
            h->n[0] = n[0]; h->n[1] = n[1]; h->n[2] = n[2];
        }
    }
    if (sc->has_room) {
        double t, n[3];
        uint32_t wall;
        if (hit_room(sc, o, d, &t, n, &wall) && t < h->t) {
            h->t = t; h->prim = wall;
            h->n[0] = n[0]; h->n[1] = n[1]; h->n[2] = n[2];
        }
    }
    return h->prim != O_MISS;
}

int o_closest_hit(const o_scene *sc, const double *o, const double *d, double tmax, double *out)
{
    o_hit h;
    int r = closest_hit(sc, o, d, tmax, &h);
    out[0] = h.t; out[1] = (double)h.prim;
    out[2] = h.n[0]; out[3] = h.n[1]; out[4] = h.n[2];
    return r;
}

static void material(const o_scene *sc, uint32_t prim, double *alb, double *emit)
{
    if (prim < (uint32_t)sc->n_prims) {
        const double *rec = sc->prims + 16 * (size_t)prim;
        for (int i = 0; i < 3; ++i) { alb[i] = rec[8 + i]; emit[i] = rec[12 + i]; }
    } else {
        for (int i = 0; i < 3; ++i) { alb[i] = sc->wall_albedo[i]; emit[i] = sc->wall_emit[i]; }
    }
}

/* specular weight k_s and GGX roughness of a primitive (record slots 11 and
 * 15); walls and diffuse scenes have none */
static void spec_of(const o_scene *sc, uint32_t prim, double *ks, double *a)
{
    *ks = 0.0;
    *a = 1.0;
    if (sc->glossy && prim < (uint32_t)sc->n_prims) {
        const double *rec = sc->prims + 16 * (size_t)prim;
        *ks = rec[11];
        *a = rec[15];
    }
}

/* Primary-vertex sampling picks the glossy lobe with probability
 * k_s / (k_s + lum(rho)) and the cosine lobe otherwise (one-sample mixture
 * of the whole BSDF, Sec. 3.3: p_1 is proportional to the entire BSDF). */
static double p_gloss(const double *rho, double ks)
{
    return ks > 0.0 ? ks / (ks + lum(rho)) : 0.0;
}

/* density of the mixture, solid angle */
static double mix_pdf(const double *rho, double ks, double a, const double *n, const double *wo, const double *wi)
{
    double pg = p_gloss(rho, ks), c = dot3(n, wi);
    double pd = c > 0.0 ? c / O_PI : 0.0;
    return (1.0 - pg) * pd + (pg > 0.0 ? pg * ggx_pdf(n, wo, wi, a) : 0.0);
}

/* full BSDF f = rho/pi + k_s f_g(wo, wi) (RGB) */
static void bsdf(const double *rho, double ks, double a, const double *n, const double *wo, const double *wi,
                 double *f)
{
    double g = ks > 0.0 ? ks * ggx_eval(n, wo, wi, a) : 0.0;
    for (int c = 0; c < 3; ++c) f[c] = rho[c] / O_PI + g;
}

/* Mutual visibility V(a, b) of two surface points (each lifted by eps along its
 * normal), or of a surface point a and the sky in direction b when b_is_dir. */
int o_visible(const o_scene *sc, const double *a, const double *na, const double *b,
              const double *nb, int b_is_dir)
{
    double o[3], d[3], tmax;
    for (int i = 0; i < 3; ++i) o[i] = a[i] + sc->eps * na[i];
    if (b_is_dir) {
        for (int i = 0; i < 3; ++i) d[i] = b[i];
        tmax = O_INF;
    } else {
        for (int i = 0; i < 3; ++i) d[i] = b[i] + sc->eps * nb[i] - o[i];
        tmax = sqrt(dot3(d, d));
        for (int i = 0; i < 3; ++i) d[i] /= tmax;
    }
    o_hit h;
    return !closest_hit(sc, o, d, tmax, &h);
}

/* ---------------------------------------------------------------------------
 * Primary vertices (step 1's starting point, Sec. 3.1): one pinhole ray
 * through each pixel centre; pixel (i, j) has index j*W + i, row 0 at the top.
 * ------------------------------------------------------------------------- */
static void camera_ray(const o_camera *c, int i, int j, double *d)
{
    double aspect = (double)c->width / (double)c->height;
    double sx = (2.0 * (i + 0.5) / c->width - 1.0) * c->tan_half_fovy * aspect;
    double sy = (1.0 - 2.0 * (j + 0.5) / c->height) * c->tan_half_fovy;
    for (int a = 0; a < 3; ++a) d[a] = c->fwd[a] + sx * c->right[a] + sy * c->up[a];
    normalize3(d);
}

void o_gbuffer(const o_scene *sc, const o_camera *cam, const int32_t *pix, int64_t npix, double *gb)
{
    int64_t total = (int64_t)cam->width * cam->height;
    int64_t n = pix ? npix : total;
    O_PARALLEL
    for (int64_t q = 0; q < n; ++q) {
        int64_t p = pix ? pix[q] : q;
        int i = (int)(p % cam->width), j = (int)(p / cam->width);
        double d[3];
        camera_ray(cam, i, j, d);
        double *g = gb + GB_N * p;
        o_hit h;
        memset(g, 0, sizeof(double) * GB_N);
        if (!closest_hit(sc, cam->eye, d, O_INF, &h)) {
            for (int a = 0; a < 3; ++a) g[GB_EMIT + a] = sc->sky[a];
            g[GB_PRIM] = (double)O_MISS;
            continue;
        }
        for (int a = 0; a < 3; ++a) {
            g[GB_POS + a] = cam->eye[a] + h.t * d[a];
            g[GB_NRM + a] = h.n[a];
        }
        material(sc, h.prim, g + GB_ALB, g + GB_EMIT);
        g[GB_DEPTH] = h.t * dot3(d, cam->fwd);
        g[GB_PRIM] = (double)h.prim;
    }
}

/* ---------------------------------------------------------------------------
 * Octahedral parameterisation (Cigolle et al. 2014) of gutter-padded square
 * tiles: N x N interior texels, one gutter texel on every side.
 * ------------------------------------------------------------------------- */
void o_oct_encode(const double *v, double *uv)
{
    double l1 = fabs(v[0]) + fabs(v[1]) + fabs(v[2]);
    double px = v[0] / l1, py = v[1] / l1;
    if (v[2] < 0.0) {
        double fx = (1.0 - fabs(py)) * sgn(px);
        double fy = (1.0 - fabs(px)) * sgn(py);
        px = fx; py = fy;
    }
    uv[0] = 0.5 * (px + 1.0);
    uv[1] = 0.5 * (py + 1.0);
}

void o_oct_decode(const double *uv, double *v)
{
    double px = 2.0 * uv[0] - 1.0, py = 2.0 * uv[1] - 1.0;
    double z = 1.0 - fabs(px) - fabs(py);
    if (z < 0.0) {
        double fx = (1.0 - fabs(py)) * sgn(px);
        double fy = (1.0 - fabs(px)) * sgn(py);
        px = fx; py = fy;
    }
    v[0] = px; v[1] = py; v[2] = z;
    normalize3(v);
}

/* IEEE binary16 rounding (nearest, ties to even) of a double, returned as a
 * double: the storage precision of a binary16 probe volume's texels.  11
 * significant bits for |x| >= 2^-14, steps of 2^-24 below (subnormals),
 * infinity from 65520 up (the tie between 65504 and 2^16 goes to the even
 * 2^16, which overflows). */
double o_round_half(double x)
{
    if (!(fabs(x) > 0.0) || !isfinite(x)) return x;
    double a = fabs(x);
    int e;
    frexp(a, &e);                                     /* a in [2^(e-1), 2^e) */
    double ulp = a >= ldexp(1.0, -14) ? ldexp(1.0, e - 11) : ldexp(1.0, -24);
    double r = nearbyint(a / ulp) * ulp;              /* exact scaling; ties to even */
    if (r > 65504.0) r = INFINITY;
    return copysign(r, x);
}

/* bilinear fetch of a padded tile with C channels at the direction v */
static void tile_fetch(const double *tile, int N, int C, const double *v, double *out)
{
    double uv[2];
    o_oct_encode(v, uv);
    int P = N + 2;
    double fx = uv[0] * N + 0.5, fy = uv[1] * N + 0.5;
    int x0 = (int)floor(fx), y0 = (int)floor(fy);
    double ax = fx - x0, ay = fy - y0;
    for (int c = 0; c < C; ++c) out[c] = 0.0;
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            double w = (dx ? ax : 1.0 - ax) * (dy ? ay : 1.0 - ay);
            const double *t = tile + C * ((size_t)(y0 + dy) * P + (x0 + dx));
            for (int c = 0; c < C; ++c) out[c] += w * t[c];
        }
}

void o_tile_fetch(const double *tile, int N, int C, const double *v, double *out)
{
    tile_fetch(tile, N, C, v, out);
}

/* A depth texel (mean, mean square) at its storage precision.  Binary16
 * (half != 0): the mean and the variance (mean square minus squared mean) as
 * binary16 values, the mean square rebuilt from them.  The variance is
 * rounded, not the mean square, because at 11 bits the difference of two
 * rounded squares of similar size would lose the variance.  Full precision:
 * the texel as it is. */
static void dep_texel(const double *t, double *m, int half)
{
    if (!half) {
        m[0] = t[0];
        m[1] = t[1];
        return;
    }
    double mu = o_round_half(t[0]), var = o_round_half(t[1] - t[0] * t[0]);
    m[0] = mu;
    m[1] = var + mu * mu;
}

/* an irradiance texel channel at its storage precision */
static double irr_texel(double v, int half) { return half ? o_round_half(v) : v; }

/* bilinear fetch of a depth tile, texels read at their storage precision */
static void dep_fetch(const double *tile, int N, const double *v, int half, double *out)
{
    double uv[2];
    o_oct_encode(v, uv);
    int P = N + 2;
    double fx = uv[0] * N + 0.5, fy = uv[1] * N + 0.5;
    int x0 = (int)floor(fx), y0 = (int)floor(fy);
    double ax = fx - x0, ay = fy - y0;
    out[0] = out[1] = 0.0;
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            double w = (dx ? ax : 1.0 - ax) * (dy ? ay : 1.0 - ay), m[2];
            dep_texel(tile + 2 * ((size_t)(y0 + dy) * P + (x0 + dx)), m, half);
            out[0] += w * m[0];
            out[1] += w * m[1];
        }
}

/* the same fetch of an irradiance tile, whose texels are read at the
 * storage precision whatever the caller's tile holds */
static void irr_fetch(const double *tile, int N, const double *v, int half, double *out)
{
    double uv[2];
    o_oct_encode(v, uv);
    int P = N + 2;
    double fx = uv[0] * N + 0.5, fy = uv[1] * N + 0.5;
    int x0 = (int)floor(fx), y0 = (int)floor(fy);
    double ax = fx - x0, ay = fy - y0;
    for (int c = 0; c < 3; ++c) out[c] = 0.0;
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            double w = (dx ? ax : 1.0 - ax) * (dy ? ay : 1.0 - ay);
            const double *t = tile + 3 * ((size_t)(y0 + dy) * P + (x0 + dx));
            for (int c = 0; c < 3; ++c) out[c] += w * irr_texel(t[c], half);
        }
}

/* Gutter fill: a border texel repeats the interior texel mirrored along its
 * edge; a corner repeats the diagonally opposite interior corner.  This makes
 * bilinear filtering continuous across the octahedral folds. */
static void fill_gutter(double *tile, int N, int C)
{
    int P = N + 2;
#define T(x, y) (tile + C * ((size_t)(y) * P + (x)))
    for (int x = 1; x <= N; ++x) {
        memcpy(T(x, 0), T(N + 1 - x, 1), sizeof(double) * C);
        memcpy(T(x, N + 1), T(N + 1 - x, N), sizeof(double) * C);
    }
    for (int y = 1; y <= N; ++y) {
        memcpy(T(0, y), T(1, N + 1 - y), sizeof(double) * C);
        memcpy(T(N + 1, y), T(N, N + 1 - y), sizeof(double) * C);
    }
    memcpy(T(0, 0), T(N, N), sizeof(double) * C);
    memcpy(T(N + 1, 0), T(1, N), sizeof(double) * C);
    memcpy(T(0, N + 1), T(N, 1), sizeof(double) * C);
    memcpy(T(N + 1, N + 1), T(1, 1), sizeof(double) * C);
#undef T
}

void o_fill_gutter(double *tile, int N, int C) { fill_gutter(tile, N, C); }

/* ---------------------------------------------------------------------------
 * Probe query Q(p, n) = E(p, n) / pi, the DDGI irradiance cache the paper
 * builds on (Sec. 2 and Eq. 4): blend of the 8 probes of p's grid cell with
 * weight = trilinear x smooth backface x Chebyshev visibility from the probe's
 * depth moments (mean visibility distance, Sec. 3.2), normalised.
 * flags bit 0 disables the backface term, bit 1 the visibility term.
 * ------------------------------------------------------------------------- */
static void probe_pos(const o_probes *pr, const int *idx, double *P)
{
    for (int a = 0; a < 3; ++a) P[a] = pr->lo[a] + (idx[a] + 0.5) * pr->spacing[a];
}

static void probe_query(const o_probes *pr, const double *p, const double *n, int flags, double *out)
{
    int base[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double g = (p[a] - pr->lo[a]) / pr->spacing[a] - 0.5;
        g = fmin(fmax(g, 0.0), (double)(pr->dims[a] - 1));
        int b = (int)floor(g);
        if (b > pr->dims[a] - 2) b = pr->dims[a] - 2;
        if (b < 0) b = 0;
        base[a] = b;
        f[a] = pr->dims[a] >= 2 ? g - b : 0.0;
    }
    int Ni = pr->irr_res, Nd = pr->dep_res;
    size_t irr_tile = (size_t)(Ni + 2) * (Ni + 2) * 3, dep_tile = (size_t)(Nd + 2) * (Nd + 2) * 2;
    double sum[3] = {0, 0, 0}, wsum = 0.0;
    for (int c = 0; c < 8; ++c) {
        int off[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1}, idx[3];
        double tri = 1.0;
        for (int a = 0; a < 3; ++a) {
            idx[a] = base[a] + off[a];
            if (idx[a] > pr->dims[a] - 1) idx[a] = pr->dims[a] - 1;
            tri *= off[a] ? f[a] : 1.0 - f[a];
        }
        size_t pi = (size_t)idx[0] + (size_t)pr->dims[0] * ((size_t)idx[1] + (size_t)pr->dims[1] * idx[2]);
        double P[3];
        probe_pos(pr, idx, P);
        double to_probe[3] = {P[0] - p[0], P[1] - p[1], P[2] - p[2]};
        double r = sqrt(dot3(to_probe, to_probe));
        double back = 0.45, vis = 1.0;
        if (r > 0.0) {
            double w[3] = {to_probe[0] / r, to_probe[1] / r, to_probe[2] / r};
            double h = 0.5 * (1.0 + dot3(n, w));
            back = h * h + 0.2;
            double from_probe[3] = {-w[0], -w[1], -w[2]}, mom[2];
            dep_fetch(pr->dep + pi * dep_tile, Nd, from_probe, pr->texel, mom);
            if (r > mom[0]) {
                double var = fmax(mom[1] - mom[0] * mom[0], pr->var_floor);
                double dd = r - mom[0];
                double cheb = var / (var + dd * dd);
                vis = cheb * cheb * cheb;
            }
        }
        if (flags & 1) back = 1.0;
        if (flags & 2) vis = 1.0;
        double w = tri * fmax(back * vis, 1e-6);
        double irr[3];
        irr_fetch(pr->irr + pi * irr_tile, Ni, n, pr->texel, irr);
        for (int a = 0; a < 3; ++a) sum[a] += w * irr[a];
        wsum += w;
    }
    for (int a = 0; a < 3; ++a) out[a] = sum[a] / wsum;
}

void o_probe_query(const o_probes *pr, int64_t n, const double *p, const double *nrm, int flags, double *out)
{
    for (int64_t i = 0; i < n; ++i) probe_query(pr, p + 3 * i, nrm + 3 * i, flags, out + 3 * i);
}

/* View-path self-shadow bias (Sec. 3.4): the query point for a surface point
 * y reached from x is moved back along the path toward x by min(d, |x-y|/2),
 * so it never crosses a surface. */
void o_view_bias(const double *y, const double *x, double d, double *out)
{
    double v[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    double dist = sqrt(dot3(v, v));
    double s = fmin(d, 0.5 * dist);
    for (int a = 0; a < 3; ++a) out[a] = y[a] + s * v[a] / dist;
}

/* ---------------------------------------------------------------------------
 * Learned cache: the MLP of oracle/mlp_ref.py written out in plain loops
 * (encoding, 78-64-64-64-64-3 with ReLU).  prec 1 rounds every GEMM operand
 * (encoded input, weights, hidden activations) to BF16 through FP32, nearest
 * even.  The output approximates E/pi like the probe query.
 * ------------------------------------------------------------------------- */
static double bf16r(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

void o_mlp_forward(const double *params, int prec, const double *lo, const double *hi, const double *pos,
                   const double *nrm, double *out)
{
    static const int dims[6] = {78, 64, 64, 64, 64, 3};
    double a[80], b[80];
    double v[6];
    for (int i = 0; i < 3; ++i) {
        v[i] = (pos[i] - lo[i]) / (hi[i] - lo[i]);
        v[3 + i] = nrm[i];
    }
    for (int i = 0; i < 6; ++i) {
        a[13 * i] = v[i];
        for (int j = 0; j < 6; ++j) {
            double f = ldexp(1.0, j) * O_PI * v[i];
            a[13 * i + 1 + 2 * j] = sin(f);
            a[13 * i + 2 + 2 * j] = cos(f);
        }
    }
    const double *w = params;
    for (int l = 0; l < 5; ++l) {
        int ni = dims[l], no = dims[l + 1];
        const double *W = w, *bias = w + ni * no;
        for (int o = 0; o < no; ++o) {
            double acc = 0.0;
            for (int k = 0; k < ni; ++k) {
                double x = prec ? bf16r(a[k]) : a[k];
                double wk = prec ? bf16r(W[o * ni + k]) : W[o * ni + k];
                acc += x * wk;
            }
            acc += bias[o];
            b[o] = (l < 4 && acc < 0.0) ? 0.0 : acc;
        }
        memcpy(a, b, sizeof(double) * no);
        w += ni * no + no;
    }
    for (int c = 0; c < 3; ++c) out[c] = a[c];
}

/* Glossy part of L_DDGI+ (Eq. 6) at a surface point: (1/2pi) times the
 * integral of E(p, wi) f_g(wo, wi) cos(theta_i) over wi, estimated with one
 * direction wi drawn from the glossy lobe (u0, u1): (1/2pi) E(p, wi) f_g cos / pdf.
 * The probes store E/pi, so E(p, wi)/(2 pi) = Q(p, wi)/2, where Q(p, wi) is the
 * probe query with the direction wi in place of the normal (the irradiance
 * read as cosine-prefiltered radiance). */
static void glossy_term(const o_probes *pr, const double *pb, const double *n, const double *wo, double ks,
                        double a, double u0, double u1, double *out)
{
    out[0] = out[1] = out[2] = 0.0;
    double wi[3];
    if (!ggx_sample(n, wo, a, u0, u1, wi)) return;
    double pdf = ggx_pdf(n, wo, wi, a);
    if (!(pdf > 0.0)) return;
    double w = ks * ggx_eval(n, wo, wi, a) * dot3(n, wi) / pdf;
    double q[3];
    probe_query(pr, pb, wi, 0, q);
    for (int c = 0; c < 3; ++c) out[c] = 0.5 * w * q[c];
}

void o_glossy_term(const o_probes *pr, const double *pb, const double *n, const double *wo, double ks, double a,
                   double u0, double u1, double *out)
{
    glossy_term(pr, pb, n, wo, ks, a, u0, u1, out);
}

/* Radiance leaving surface point y toward x: L_e(y) + rho_y * C(y), the
 * radiance L_DDGI+ of Eq. 4/5 (diffuse term rho/pi * E = rho * E/pi).  C is
 * the probe query Q(y_b, n_y) at the view-path-biased point, or, when a
 * learned cache is set and allowed, its output max(0, MLP(y, n_y)) at y
 * itself (the bias only guards the probes' visibility test).  A surface with
 * a specular layer adds the glossy part of Eq. 6 (one lobe sample, uniforms
 * ug) at the same biased point; ug = NULL leaves it out. */
static void radiance_toward_ex(const o_scene *sc, const o_probes *pr, uint32_t prim, const double *y,
                               const double *ny, const double *x, int allow_mlp, const double *ug, double *L)
{
    double alb[3], emit[3], ks, ra;
    material(sc, prim, alb, emit);
    spec_of(sc, prim, &ks, &ra);
    for (int a = 0; a < 3; ++a) L[a] = emit[a];
    int diffuse = alb[0] != 0.0 || alb[1] != 0.0 || alb[2] != 0.0;
    if (diffuse) {
        double q[3];
        if (allow_mlp && pr->mlp) {
            o_mlp_forward(pr->mlp, pr->mlp_prec, pr->mlp_lo, pr->mlp_hi, y, ny, q);
            for (int a = 0; a < 3; ++a) q[a] = fmax(q[a], 0.0);
        } else {
            double pb[3];
            o_view_bias(y, x, pr->bias_dist, pb);
            probe_query(pr, pb, ny, 0, q);
        }
        for (int a = 0; a < 3; ++a) L[a] += alb[a] * q[a];
    }
    if (ks > 0.0 && ug) {
        double pb[3], wo[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]}, g[3];
        normalize3(wo);
        o_view_bias(y, x, pr->bias_dist, pb);
        glossy_term(pr, pb, ny, wo, ks, ra, ug[0], ug[1], g);
        for (int a = 0; a < 3; ++a) L[a] += g[a];
    }
}

static void radiance_toward(const o_scene *sc, const o_probes *pr, uint32_t prim, const double *y,
                            const double *ny, const double *x, double *L)
{
    radiance_toward_ex(sc, pr, prim, y, ny, x, 1, NULL, L);
}

/* ---------------------------------------------------------------------------
 * Probe update (Eq. 5, Sec. 3.2): each probe traces R uniform-sphere rays;
 * a ray that hits h brings L_e(h) + rho_h Q_prev(h_b, n_h) (single-bounce
 * recursion, emission not diffused), a ray that leaves brings the sky.
 * Irradiance texel with centre direction n_t takes the cosine-weighted mean
 * sum max(0, n_t.w) L / sum max(0, n_t.w), which estimates E/pi; depth texel
 * takes the max(0, n_t.w)^sharpness weighted mean of (d, d^2), d = min(t, d_max).
 * Stored = hysteresis * old + (1 - hysteresis) * new; then gutters.
 * Q_prev is read from the input textures only.
 * ------------------------------------------------------------------------- */
void o_probe_update(const o_scene *sc, const o_probes *in, double *irr_out, double *dep_out,
                    int rays, double hysteresis, double sharpness, double slider, uint64_t seed,
                    uint32_t frame, const int32_t *plist, int64_t nlist)
{
    int Ni = in->irr_res, Nd = in->dep_res;
    int64_t P = (int64_t)in->dims[0] * in->dims[1] * in->dims[2];
    size_t irr_tile = (size_t)(Ni + 2) * (Ni + 2) * 3, dep_tile = (size_t)(Nd + 2) * (Nd + 2) * 2;
    int64_t n = plist ? nlist : P;
    if (rays > 4096) rays = 4096;
    O_PARALLEL
    for (int64_t q = 0; q < n; ++q) {
        double (*dirs)[3] = malloc(sizeof(double) * 3 * (size_t)rays);
        double (*Ls)[3] = malloc(sizeof(double) * 3 * (size_t)rays);
        double *ds = malloc(sizeof(double) * (size_t)rays);
        int64_t pi = plist ? plist[q] : q;
        int idx[3] = {(int)(pi % in->dims[0]), (int)((pi / in->dims[0]) % in->dims[1]),
                      (int)(pi / ((int64_t)in->dims[0] * in->dims[1]))};
        double Pp[3];
        probe_pos(in, idx, Pp);
        for (int r = 0; r < rays; ++r) {
            double u[4];
            rand4(seed, (uint32_t)pi, frame, PASS_PROBE, (uint32_t)r, u);
            o_sphere_dir(u[0], u[1], dirs[r]);
            o_hit h;
            if (closest_hit(sc, Pp, dirs[r], O_INF, &h)) {
                double hp[3], alb[3], emit[3];
                for (int a = 0; a < 3; ++a) hp[a] = Pp[a] + h.t * dirs[r][a];
                material(sc, h.prim, alb, emit);
                if (slider > 0.0 && (emit[0] != 0.0 || emit[1] != 0.0 || emit[2] != 0.0)) {
                    /* distance heuristic (Sec. 3.2): the surfaces this probe shades lie
                     * behind it; their distance to the light is estimated as the ray
                     * length t plus the probe's own mean depth in the backward
                     * direction, clipped to the probe's cell; emission is scaled by the
                     * inverse square of that total relative to t, with the backward
                     * part weighted by the per-scene slider */
                    double back[3] = {-dirs[r][0], -dirs[r][1], -dirs[r][2]}, mom[2];
                    dep_fetch(in->dep + pi * dep_tile, Nd, back, in->texel, mom);
                    double clip = O_INF;
                    for (int a = 0; a < 3; ++a)
                        if (back[a] != 0.0) clip = fmin(clip, 0.5 * in->spacing[a] / fabs(back[a]));
                    double db = fmin(fmax(mom[0], 0.0), clip);
                    double ratio = h.t / (h.t + slider * db);
                    for (int a = 0; a < 3; ++a) emit[a] *= ratio * ratio;
                }
                for (int a = 0; a < 3; ++a) Ls[r][a] = emit[a];
                if (alb[0] != 0.0 || alb[1] != 0.0 || alb[2] != 0.0) {
                    double hb[3], qv[3];
                    o_view_bias(hp, Pp, in->bias_dist, hb);
                    probe_query(in, hb, h.n, 0, qv);
                    for (int a = 0; a < 3; ++a) Ls[r][a] += alb[a] * qv[a];
                }
                double ks, ra;
                spec_of(sc, h.prim, &ks, &ra);
                if (ks > 0.0) {
                    /* L_DDGI+ with its glossy part (Eq. 6) toward the probe */
                    double hb[3], ug[4], wo[3] = {-dirs[r][0], -dirs[r][1], -dirs[r][2]}, gq[3];
                    o_view_bias(hp, Pp, in->bias_dist, hb);
                    rand4(seed, (uint32_t)pi, frame, PASS_GLOSSY_PROBE, (uint32_t)r, ug);
                    glossy_term(in, hb, h.n, wo, ks, ra, ug[0], ug[1], gq);
                    for (int a = 0; a < 3; ++a) Ls[r][a] += gq[a];
                }
                ds[r] = fmin(h.t, in->d_max);
            } else {
                for (int a = 0; a < 3; ++a) Ls[r][a] = sc->sky[a];
                ds[r] = in->d_max;
            }
        }
        const double *iold = in->irr + pi * irr_tile;
        const double *dold = in->dep + pi * dep_tile;
        double *inew = irr_out + pi * irr_tile;
        double *dnew = dep_out + pi * dep_tile;
        for (int ty = 0; ty < Ni; ++ty)
            for (int tx = 0; tx < Ni; ++tx) {
                double uv[2] = {(tx + 0.5) / Ni, (ty + 0.5) / Ni}, nt[3];
                o_oct_decode(uv, nt);
                double num[3] = {0, 0, 0}, den = 0.0;
                for (int r = 0; r < rays; ++r) {
                    double w = fmax(0.0, dot3(nt, dirs[r]));
                    for (int a = 0; a < 3; ++a) num[a] += w * Ls[r][a];
                    den += w;
                }
                size_t o = 3 * ((size_t)(ty + 1) * (Ni + 2) + (tx + 1));
                for (int a = 0; a < 3; ++a) {
                    const double old = irr_texel(iold[o + a], in->texel);
                    double nv = den > 0.0 ? num[a] / den : old;
                    /* stored at the storage precision, blended from the stored old texel */
                    inew[o + a] = irr_texel(hysteresis * old + (1.0 - hysteresis) * nv, in->texel);
                }
            }
        for (int ty = 0; ty < Nd; ++ty)
            for (int tx = 0; tx < Nd; ++tx) {
                double uv[2] = {(tx + 0.5) / Nd, (ty + 0.5) / Nd}, nt[3];
                o_oct_decode(uv, nt);
                double m1 = 0.0, m2 = 0.0, den = 0.0;
                for (int r = 0; r < rays; ++r) {
                    double w = pow(fmax(0.0, dot3(nt, dirs[r])), sharpness);
                    m1 += w * ds[r];
                    m2 += w * ds[r] * ds[r];
                    den += w;
                }
                size_t o = 2 * ((size_t)(ty + 1) * (Nd + 2) + (tx + 1));
                /* blended from the stored old texel, stored at the storage
                 * precision (binary16: as (mean, variance)) and kept here as
                 * (mean, mean square) */
                double old[2], b[2];
                dep_texel(dold + o, old, in->texel);
                double n1 = den > 0.0 ? m1 / den : old[0];
                double n2 = den > 0.0 ? m2 / den : old[1];
                b[0] = hysteresis * old[0] + (1.0 - hysteresis) * n1;
                b[1] = hysteresis * old[1] + (1.0 - hysteresis) * n2;
                dep_texel(b, dnew + o, in->texel);
            }
        fill_gutter(inew, Ni, 3);
        fill_gutter(dnew, Nd, 2);
        free(dirs);
        free(Ls);
        free(ds);
    }
}

/* ---------------------------------------------------------------------------
 * Target function and reuse helpers
 * ------------------------------------------------------------------------- */
/* p_hat at shading point (x, n_x, rho_x) for a reservoir sample: the
 * luminance of the bounded-geometry contribution rho_x/pi * L(y) * min(G, G_max)
 * (Sec. 3.1 step 2 and Sec. 3.5), using the sample's cached radiance
 * (query caching, Sec. 3.6).  Sky samples (zero n_y) use G := cos(theta_x). */
static double target(const double *x, const double *nx, const double *rho, const double *y,
                     const double *ny, const double *L, double g_max)
{
    double f[3] = {rho[0] / O_PI * L[0], rho[1] / O_PI * L[1], rho[2] / O_PI * L[2]};
    if (ny[0] == 0.0 && ny[1] == 0.0 && ny[2] == 0.0) {
        double cx = dot3(nx, y);
        return cx > 0.0 ? lum(f) * cx : 0.0;
    }
    double v[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
    double d2 = dot3(v, v), d = sqrt(d2);
    double w[3] = {v[0] / d, v[1] / d, v[2] / d};
    double cx = dot3(nx, w), cy = -dot3(ny, w);
    if (cx <= 0.0 || cy <= 0.0) return 0.0;
    double G = cx * cy / d2;
    return lum(f) * fmin(G, g_max);
}

/* The same with the full BSDF of a glossy scene: f(x, wo, wi) = rho/pi +
 * k_s f_g(wo, wi), wo toward the camera at eye, wi toward the sample. */
static double target_glossy(const o_scene *sc, const double *g, const double *eye, const double *y,
                            const double *ny, const double *L, double g_max)
{
    const double *x = g + GB_POS, *nx = g + GB_NRM, *rho = g + GB_ALB;
    double ks, a, f[3], wo[3] = {eye[0] - x[0], eye[1] - x[1], eye[2] - x[2]};
    spec_of(sc, (uint32_t)g[GB_PRIM], &ks, &a);
    normalize3(wo);
    if (ny[0] == 0.0 && ny[1] == 0.0 && ny[2] == 0.0) {
        double cx = dot3(nx, y);
        if (cx <= 0.0) return 0.0;
        bsdf(rho, ks, a, nx, wo, y, f);
        double fl[3] = {f[0] * L[0], f[1] * L[1], f[2] * L[2]};
        return lum(fl) * cx;
    }
    double v[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
    double d2 = dot3(v, v), d = sqrt(d2);
    double w[3] = {v[0] / d, v[1] / d, v[2] / d};
    double cx = dot3(nx, w), cy = -dot3(ny, w);
    if (cx <= 0.0 || cy <= 0.0) return 0.0;
    bsdf(rho, ks, a, nx, wo, w, f);
    double fl[3] = {f[0] * L[0], f[1] * L[1], f[2] * L[2]};
    return lum(fl) * fmin(cx * cy / d2, g_max);
}

static double res_target(const o_scene *sc, const double *g, const double *eye, const double *r, double g_max)
{
    if (sc->glossy) return target_glossy(sc, g, eye, r + R_Y, r + R_NY, r + R_L, g_max);
    return target(g + GB_POS, g + GB_NRM, g + GB_ALB, r + R_Y, r + R_NY, r + R_L, g_max);
}

static int res_is_sky(const double *r)
{
    return r[R_NY] == 0.0 && r[R_NY + 1] == 0.0 && r[R_NY + 2] == 0.0;
}

/* a pixel is shaded when its surface reflects: diffuse albedo or a specular layer */
static int pixel_active(const o_scene *sc, const double *g)
{
    if ((uint32_t)g[GB_PRIM] == O_MISS) return 0;
    if (g[GB_ALB] != 0.0 || g[GB_ALB + 1] != 0.0 || g[GB_ALB + 2] != 0.0) return 1;
    double ks, a;
    spec_of(sc, (uint32_t)g[GB_PRIM], &ks, &a);
    return ks > 0.0;
}

static void res_empty(double *r, double M)
{
    memset(r, 0, sizeof(double) * R_N);
    r[R_M] = M;
    r[R_TAG] = (double)0xFFFFFFFFu;
    r[R_PRIM] = (double)O_MISS;
}

static double make_tag(int64_t pixel, int cand, uint32_t frame)
{
    uint32_t t = ((uint32_t)(pixel & 0x7FFFFF) << 9) | ((uint32_t)(cand & 31) << 4) | (frame & 15u);
    return (double)t;
}

/* geometric similarity test used by temporal and spatial reuse */
static int similar(const double *g, const double *gq, const o_params *pp)
{
    if ((uint32_t)gq[GB_PRIM] == O_MISS) return 0;
    if (dot3(g + GB_NRM, gq + GB_NRM) < pp->cos_n) return 0;
    if (fabs(g[GB_DEPTH] - gq[GB_DEPTH]) > pp->depth_rel * g[GB_DEPTH]) return 0;
    return 1;
}

/* ---------------------------------------------------------------------------
 * Initial resampling (Sec. 3.1 steps 1-2, Fig. 2; Sec. 3.5; Sec. 3.6):
 * M cosine-sampled candidates y_i, converted to area measure, streamed
 * through a weighted reservoir with w_i = p_hat(y_i) / p_A(y_i), where
 * p_A = cos(theta_x)/pi * cos(theta_y)/|x-y|^2.  The reservoir keeps the
 * sample's radiance L(y) (the cached query).  The residual transport with
 * the unbounded part max(0, G - G_max) is estimated from candidate 0 (the
 * auxiliary BSDF sample of Sec. 3.5, Eq. 9).
 * Replacement rule: candidate i replaces the current sample iff
 * u_2 * wsum < w_i after wsum has been increased by w_i.
 * Emitter samples (Sec. 3.1 step 1 draws candidates from the BSDF and from
 * the emitters; Fig. 2 selects them in proportion to L_e + L_DDGI): M_light
 * more candidates i = M .. M+M_light-1, each a point uniform in the area of
 * an emissive sphere chosen uniformly (u0 the sphere, u1, u2 the point, u3
 * the reservoir decision).  With both techniques every candidate's weight is
 * p_hat over the balance-heuristic mixture density (M p_bsdf + M_light
 * p_light) / (M + M_light) in area measure, and the reservoir counts all
 * M + M_light candidates; with M_light = 0 this is the weight above.  The
 * density of cosine sampling is taken without visibility: a light sample
 * that x cannot see has zero contribution, so its weight does not matter.
 * ------------------------------------------------------------------------- */
/* Emitters for light sampling: the emissive spheres, in index order. */
static int emitter_list(const o_scene *sc, int32_t *out, int cap)
{
    int n = 0;
    for (int32_t i = 0; i < sc->n_prims; ++i) {
        const double *rec = sc->prims + 16 * i;
        if ((int)rec[3] == 0 && (rec[12] > 0.0 || rec[13] > 0.0 || rec[14] > 0.0) && n < cap) out[n++] = i;
    }
    return n;
}

/* area-measure density of the emitter technique at a point of primitive prim */
static double light_pdf(const o_scene *sc, const int32_t *em, int n_em, uint32_t prim)
{
    for (int e = 0; e < n_em; ++e)
        if ((uint32_t)em[e] == prim) {
            double r = sc->prims[16 * em[e] + 4];
            return 1.0 / ((double)n_em * 4.0 * O_PI * r * r);
        }
    return 0.0;
}

void o_resample_initial(const o_scene *sc, int32_t W, int32_t H, const double *gb, const o_probes *pr,
                        const o_params *pp, uint64_t seed, uint32_t frame, const int32_t *pix,
                        int64_t npix, double *res, double *resid)
{
    int32_t em[256];
    const int n_em = pp->M_light > 0 ? emitter_list(sc, em, 256) : 0;
    const int Mb = pp->M, Ml = pp->M_light, Mt = Mb + Ml;
    int64_t n = pix ? npix : (int64_t)W * H;
    O_PARALLEL
    for (int64_t q = 0; q < n; ++q) {
        int64_t p = pix ? pix[q] : q;
        const double *g = gb + GB_N * p;
        double *r = res + R_N * p, *rs = resid + 3 * p;
        rs[0] = rs[1] = rs[2] = 0.0;
        if (!pixel_active(sc, g)) { res_empty(r, 0.0); continue; }
        const double *x = g + GB_POS, *nx = g + GB_NRM, *rho = g + GB_ALB;
        double o[3];
        for (int a = 0; a < 3; ++a) o[a] = x[a] + sc->eps * nx[a];
        /* glossy scene: the whole BSDF at x, wo toward the camera (Sec. 3.3) */
        double ks_x = 0.0, a_x = 1.0, pg_x = 0.0, wo_x[3] = {0.0, 0.0, 1.0};
        if (sc->glossy) {
            spec_of(sc, (uint32_t)g[GB_PRIM], &ks_x, &a_x);
            pg_x = p_gloss(rho, ks_x);
            for (int a = 0; a < 3; ++a) wo_x[a] = pp->eye[a] - x[a];
            normalize3(wo_x);
        }
        double wsum = 0.0, p_sel = 0.0;
        int have = 0;
        res_empty(r, 0.0);
        /* subsampling (Sec. 6): a pixel that draws no candidates this frame keeps an
         * empty reservoir (M = 0) and only estimates the residual from candidate 0 */
        const int draws = pp->subsample <= 1 || ((p % W) + (p / W) + (int64_t)frame) % pp->subsample == 0;
        for (int i = 0; i < (draws ? Mt : 1); ++i) {
            double u[4], w[3];
            rand4(seed, (uint32_t)p, frame, PASS_INITIAL, (uint32_t)i, u);
            double y[3], ny[3] = {0, 0, 0}, L[3], phat = 0.0, wi = 0.0;
            uint32_t prim = O_MISS;
            int surface = 0, dir_ok = 1;
            double u_dec = u[2];
            if (i < Mb) {
                /* BSDF candidate: the first surface along the ray; cosine-distributed,
                 * or in a glossy scene drawn from the glossy lobe with probability
                 * p_gloss (u3), a lobe sample below the surface giving no candidate */
                if (pg_x > 0.0 && u[3] < pg_x) dir_ok = ggx_sample(nx, wo_x, a_x, u[0], u[1], w);
                else o_cosine_dir(nx, u[0], u[1], w);
                o_hit h;
                if (dir_ok && closest_hit(sc, o, w, O_INF, &h)) {
                    for (int a = 0; a < 3; ++a) { y[a] = o[a] + h.t * w[a]; ny[a] = h.n[a]; }
                    prim = h.prim;
                    surface = 1;
                }
            } else {
                /* emitter candidate: an emitter chosen uniformly, a point uniform in its area */
                u_dec = u[3];
                if (n_em > 0) {
                    int e = (int)floor(u[0] * (double)n_em);
                    const double *rec = sc->prims + 16 * em[e];
                    double d[3];
                    o_sphere_dir(u[1], u[2], d);
                    for (int a = 0; a < 3; ++a) { y[a] = rec[a] + rec[4] * d[a]; ny[a] = d[a]; }
                    prim = (uint32_t)em[e];
                    surface = 1;
                }
            }
            if (surface) {
                double v[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
                double d2 = dot3(v, v), d = sqrt(d2);
                double wv[3] = {v[0] / d, v[1] / d, v[2] / d};
                double cx = dot3(nx, wv), cy = -dot3(ny, wv);
                if (cx > 0.0 && cy > 0.0) {
                    double G = cx * cy / d2, f[3], pA;
                    if (sc->glossy) {
                        /* f(x, wo, wi) L(y) with L_DDGI+ at y including its glossy part
                         * (one lobe sample, counter (p, frame, 14, i)); p_A from the
                         * BSDF mixture's solid-angle density */
                        double ug[4], fb[3];
                        rand4(seed, (uint32_t)p, frame, PASS_GLOSSY_CAND, (uint32_t)i, ug);
                        radiance_toward_ex(sc, pr, prim, y, ny, x, 1, ug, L);
                        bsdf(rho, ks_x, a_x, nx, wo_x, wv, fb);
                        for (int a = 0; a < 3; ++a) f[a] = fb[a] * L[a];
                        pA = mix_pdf(rho, ks_x, a_x, nx, wo_x, wv) * cy / d2;
                    } else {
                        radiance_toward(sc, pr, prim, y, ny, x, L);
                        for (int a = 0; a < 3; ++a) f[a] = rho[a] / O_PI * L[a];
                        pA = cx / O_PI * cy / d2;
                    }
                    phat = lum(f) * fmin(G, pp->g_max);
                    /* balance heuristic: p_hat over the candidates' mixture density
                     * (Mb p_bsdf + Ml p_light) / Mt, area measure */
                    if (!(pA > 0.0) && Ml == 0) wi = 0.0;
                    else if (Ml == 0) wi = phat / pA;
                    else wi = phat * Mt / (Mb * pA + Ml * light_pdf(sc, em, n_em, prim));
                    if (i == 0 && G > pp->g_max) {
                        /* residual f L (G - G_max) / p_A: for the Lambertian BSDF
                         * rho L (1 - G_max / G) */
                        if (sc->glossy)
                            for (int a = 0; a < 3; ++a) rs[a] = pA > 0.0 ? f[a] * (G - pp->g_max) / pA : 0.0;
                        else
                            for (int a = 0; a < 3; ++a) rs[a] = rho[a] * L[a] * (1.0 - pp->g_max / G);
                    }
                }
            } else if (i < Mb && dir_ok) {
                for (int a = 0; a < 3; ++a) { y[a] = w[a]; L[a] = sc->sky[a]; }
                double cx = dot3(nx, w);
                if (cx > 0.0) {
                    if (sc->glossy) {
                        double fb[3], f[3], pd = mix_pdf(rho, ks_x, a_x, nx, wo_x, w);
                        bsdf(rho, ks_x, a_x, nx, wo_x, w, fb);
                        for (int a = 0; a < 3; ++a) f[a] = fb[a] * L[a];
                        phat = lum(f) * cx;
                        wi = pd > 0.0 ? phat / pd * ((double)Mt / Mb) : 0.0;
                    } else {
                        double f[3] = {rho[0] / O_PI * L[0], rho[1] / O_PI * L[1], rho[2] / O_PI * L[2]};
                        phat = lum(f) * cx;
                        wi = phat / (cx / O_PI) * ((double)Mt / Mb);
                    }
                }
            }
            if (!draws) break;
            wsum += wi;
            if (u_dec * wsum < wi) {
                have = 1;
                p_sel = phat;
                for (int a = 0; a < 3; ++a) { r[R_Y + a] = y[a]; r[R_NY + a] = ny[a]; r[R_L + a] = L[a]; }
                r[R_TAG] = make_tag(p, i, frame);
                r[R_PRIM] = (double)prim;
            }
        }
        if (!draws) continue;
        r[R_WSUM] = wsum;
        r[R_M] = (double)Mt;
        r[R_W] = (have && p_sel > 0.0) ? wsum / (Mt * p_sel) : 0.0;
    }
}

/* ---------------------------------------------------------------------------
 * Reservoir merge shared by temporal and spatial reuse (Sec. 3.1 step 2):
 * candidate reservoir q enters with weight p_hat_x(y_q) * W_q * M_q and
 * replaces the sample iff u * wsum < w_q.  The normalisation either counts
 * the M_q of every merged domain whose own target supports the chosen y and
 * sees it (V traced from x_q), or (biased) all of them.  In the unbiased form
 * a chosen sample that x itself cannot see is dropped (W = 0, M kept).
 * ------------------------------------------------------------------------- */
typedef struct {
    double wsum, Msum;
    const double *sel;
} merge_state;

static void merge_in(const o_scene *sc, merge_state *s, const double *g, const double *eye, const double *rq,
                     double Mq, double u, double g_max)
{
    double w = 0.0;
    if (rq[R_W] > 0.0 && Mq > 0.0) w = res_target(sc, g, eye, rq, g_max) * rq[R_W] * Mq;
    s->wsum += w;
    s->Msum += Mq;
    if (u * s->wsum < w) s->sel = rq;
}

static void finish_merge(const o_scene *sc, const merge_state *s, const double *g, int ndom,
                         const double *const *gdom, const double *const *edom, const double *Mdom,
                         const o_params *pp, double *out)
{
    double tmp[R_N];
    if (!s->sel) {
        res_empty(tmp, s->Msum);
        tmp[R_WSUM] = s->wsum;
        memcpy(out, tmp, sizeof tmp);
        return;
    }
    memcpy(tmp, s->sel, sizeof tmp);
    double ph = res_target(sc, g, edom[0], tmp, pp->g_max);
    double Z;
    int keep = 1;
    if (pp->unbiased) {
        /* domain 0 is the pixel itself; a sample it cannot see is dropped so
         * that every reservoir only holds samples visible from its own pixel,
         * which is the support the next pass's normalisation assumes */
        int sky = res_is_sky(tmp);
        int vis_x = o_visible(sc, g + GB_POS, g + GB_NRM, tmp + R_Y, tmp + R_NY, sky);
        keep = vis_x;
        Z = 0.0;
        for (int j = 0; j < ndom; ++j) {
            const double *gq = gdom[j];
            if (Mdom[j] <= 0.0) continue;
            if (res_target(sc, gq, edom[j], tmp, pp->g_max) <= 0.0) continue;
            int v = j == 0 ? vis_x : o_visible(sc, gq + GB_POS, gq + GB_NRM, tmp + R_Y, tmp + R_NY, sky);
            if (!v) continue;
            Z += Mdom[j];
        }
    } else {
        Z = s->Msum;
    }
    tmp[R_WSUM] = s->wsum;
    tmp[R_M] = s->Msum;
    tmp[R_W] = (keep && Z > 0.0 && ph > 0.0) ? s->wsum / (Z * ph) : 0.0;
    memcpy(out, tmp, sizeof tmp);
}

/* Reprojection of x into a camera: continuous pixel coordinates, floor.
 * Returns the pixel index or -1 when x is behind the camera or off-screen. */
int64_t o_reproject(const o_camera *c, const double *x)
{
    double v[3] = {x[0] - c->eye[0], x[1] - c->eye[1], x[2] - c->eye[2]};
    double z = dot3(v, c->fwd);
    if (z <= 0.0) return -1;
    double aspect = (double)c->width / (double)c->height;
    double sx = dot3(v, c->right) / (z * c->tan_half_fovy * aspect);
    double sy = dot3(v, c->up) / (z * c->tan_half_fovy);
    double px = (sx + 1.0) * 0.5 * c->width, py = (1.0 - sy) * 0.5 * c->height;
    double fx = floor(px), fy = floor(py);
    if (fx < 0.0 || fy < 0.0 || fx >= c->width || fy >= c->height) return -1;
    return (int64_t)fy * c->width + (int64_t)fx;
}

/* ---------------------------------------------------------------------------
 * Temporal reuse (Sec. 3.1 step 2, "among previous frames"; Sec. 3.6 for the
 * cached radiance): merge the current reservoir with the history reservoir
 * of the pixel x lands on in the previous camera, if that pixel passes the
 * normal/depth test; the history's M is capped at floor(m_cap (M + M_light)),
 * a multiple of the per-frame candidate count.
 * ------------------------------------------------------------------------- */
void o_resample_temporal(const o_scene *sc, int32_t W, int32_t H, const double *gb, const double *gb_prev,
                         const o_camera *cam_prev, const double *cur, const double *hist,
                         const o_params *pp, uint64_t seed, uint32_t frame, const int32_t *pix,
                         int64_t npix, double *out)
{
    int64_t n = pix ? npix : (int64_t)W * H;
    O_PARALLEL
    for (int64_t q = 0; q < n; ++q) {
        int64_t p = pix ? pix[q] : q;
        const double *g = gb + GB_N * p;
        const double *rc = cur + R_N * p;
        if (!pixel_active(sc, g)) { memcpy(out + R_N * p, rc, sizeof(double) * R_N); continue; }
        merge_state s = {0.0, 0.0, NULL};
        const double *gdom[2], *edom[2];
        double Mdom[2];
        int nd = 0;
        merge_in(sc, &s, g, pp->eye, rc, rc[R_M], 0.0, pp->g_max);
        gdom[nd] = g; edom[nd] = pp->eye; Mdom[nd] = rc[R_M]; ++nd;
        int64_t pp_idx = o_reproject(cam_prev, g + GB_POS);
        if (pp_idx >= 0 && similar(g, gb_prev + GB_N * pp_idx, pp)) {
            const double *rh = hist + R_N * pp_idx;
            /* the cap is a multiple of the candidates a drawing pixel takes per
             * frame, so a pixel that drew none this frame (candidate
             * subsampling, Sec. 6) still takes over its history */
            double Mh = fmin(rh[R_M], floor(pp->m_cap * (double)(pp->M + pp->M_light)));
            double u[4];
            rand4(seed, (uint32_t)p, frame, PASS_TEMPORAL, 0u, u);
            merge_in(sc, &s, g, pp->eye, rh, Mh, u[0], pp->g_max);
            gdom[nd] = gb_prev + GB_N * pp_idx; edom[nd] = pp->eye_prev; Mdom[nd] = Mh; ++nd;
        }
        finish_merge(sc, &s, g, nd, gdom, edom, Mdom, pp, out + R_N * p);
    }
}

/* Neighbour candidate j of pixel p in spatial pass s (before validation):
 * uniform point in the disk of the given radius, rounded half up. */
int64_t o_spatial_candidate(int32_t W, int32_t H, int64_t p, int j, double radius, uint64_t seed,
                            uint32_t frame, int pass, double *u2)
{
    double u[4];
    rand4(seed, (uint32_t)p, frame, (uint32_t)(PASS_SPATIAL0 + pass), (uint32_t)j, u);
    double rad = radius * sqrt(u[0]), ang = 2.0 * O_PI * u[1];
    int64_t px = p % W, py = p / W;
    int64_t qx = px + (int64_t)floor(rad * cos(ang) + 0.5);
    int64_t qy = py + (int64_t)floor(rad * sin(ang) + 0.5);
    if (u2) *u2 = u[2];
    if (qx < 0 || qy < 0 || qx >= W || qy >= H) return -1;
    if (qx == px && qy == py) return -1;
    return qy * W + qx;
}

/* ---------------------------------------------------------------------------
 * Spatial reuse (Sec. 3.1 step 2, "among neighboring pixels"; Sec. 3.6):
 * merge the pixel's own reservoir, then k neighbours from a disk that pass
 * the normal/depth test.  Rejected neighbours are neither counted nor retried.
 * ------------------------------------------------------------------------- */
void o_resample_spatial(const o_scene *sc, int32_t W, int32_t H, const double *gb, const double *in,
                        const o_params *pp, int pass, uint64_t seed, uint32_t frame, const int32_t *pix,
                        int64_t npix, double *out)
{
    int64_t n = pix ? npix : (int64_t)W * H;
    O_PARALLEL
    for (int64_t q = 0; q < n; ++q) {
        const double *gdom[16], *edom[16];
        double Mdom[16];
        for (int j = 0; j < 16; ++j) edom[j] = pp->eye;
        int64_t p = pix ? pix[q] : q;
        const double *g = gb + GB_N * p;
        const double *rc = in + R_N * p;
        if (!pixel_active(sc, g)) { memcpy(out + R_N * p, rc, sizeof(double) * R_N); continue; }
        merge_state s = {0.0, 0.0, NULL};
        int nd = 0;
        merge_in(sc, &s, g, pp->eye, rc, rc[R_M], 0.0, pp->g_max);
        gdom[nd] = g; Mdom[nd] = rc[R_M]; ++nd;
        for (int j = 0; j < pp->k && j < 15; ++j) {
            double u2;
            int64_t qq = o_spatial_candidate(W, H, p, j, pp->radius, seed, frame, pass, &u2);
            if (qq < 0) continue;
            const double *gq = gb + GB_N * qq;
            if (!similar(g, gq, pp)) continue;
            const double *rq = in + R_N * qq;
            merge_in(sc, &s, g, pp->eye, rq, rq[R_M], u2, pp->g_max);
            gdom[nd] = gq; Mdom[nd] = rq[R_M]; ++nd;
        }
        finish_merge(sc, &s, g, nd, gdom, edom, Mdom, pp, out + R_N * p);
    }
}

/* ---------------------------------------------------------------------------
 * Shading (Sec. 3.1 steps 3-4; Eq. 9): L_o = L_e(x) + bounded term + residual,
 * bounded term = rho_x/pi * L(y; x) * min(G, G_max) * V(x, y) * W with a fresh
 * radiance query biased toward this x (the per-vertex query of Sec. 3.6) and
 * one shadow ray.  A primary ray that left the scene shows the sky.
 * ------------------------------------------------------------------------- */
/* Specular recursion for shading (Sec. 3.3, Eq. 7-8), a glossy scene's
 * radiance leaving surface point v (primitive prim, normal nv) toward the
 * previous path vertex prev: L_e(v) + rho_v Q(v_b, n_v), the diffuse part
 * always from the probes, plus the glossy part of one direction wi drawn from
 * v's glossy lobe (counter (pixel, frame, 16, depth)), weighted by
 * k_s f_g cos / pdf.  The path's footprint a(x_1 .. x_n) = (sum over its
 * segments of sqrt(|x_i - x_{i+1}|^2 / (p_i cos_{i+1})))^2, with p_i the
 * solid-angle density that chose segment i, decides: once it exceeds a_0 c,
 * or at the depth limit, the glossy integral is estimated from the probes
 * (Q(v_b, wi)/2, Eq. 6); below it the ray is traced and the recursion
 * continues at the surface it hits (the sky if it leaves).  foot_sum holds the
 * sum over the segments up to v. */
static void shade_radiance(const o_scene *sc, const o_probes *pr, const o_params *pp, uint64_t seed,
                           uint32_t pixel, uint32_t frame, uint32_t prim, const double *v, const double *nv,
                           const double *prev, double foot_sum, double a0c, int depth, double *L)
{
    double alb[3], emit[3], ks, ra, pb[3], q[3];
    material(sc, prim, alb, emit);
    spec_of(sc, prim, &ks, &ra);
    for (int a = 0; a < 3; ++a) L[a] = emit[a];
    o_view_bias(v, prev, pr->bias_dist, pb);
    if (alb[0] != 0.0 || alb[1] != 0.0 || alb[2] != 0.0) {
        probe_query(pr, pb, nv, 0, q);
        for (int a = 0; a < 3; ++a) L[a] += alb[a] * q[a];
    }
    if (!(ks > 0.0)) return;
    double wo[3] = {prev[0] - v[0], prev[1] - v[1], prev[2] - v[2]}, wi[3], u[4];
    normalize3(wo);
    rand4(seed, pixel, frame, PASS_GLOSSY_SHADE, (uint32_t)depth, u);
    if (!ggx_sample(nv, wo, ra, u[0], u[1], wi)) return;
    double pdf = ggx_pdf(nv, wo, wi, ra);
    if (!(pdf > 0.0)) return;
    double wgt = ks * ggx_eval(nv, wo, wi, ra) * dot3(nv, wi) / pdf;
    if (foot_sum * foot_sum > a0c || depth >= pp->glossy_depth) {
        probe_query(pr, pb, wi, 0, q);
        for (int a = 0; a < 3; ++a) L[a] += 0.5 * wgt * q[a];
        return;
    }
    double o[3];
    for (int a = 0; a < 3; ++a) o[a] = v[a] + sc->eps * nv[a];
    o_hit h;
    if (!closest_hit(sc, o, wi, O_INF, &h)) {
        for (int a = 0; a < 3; ++a) L[a] += wgt * sc->sky[a];
        return;
    }
    double z[3];
    for (int a = 0; a < 3; ++a) z[a] = o[a] + h.t * wi[a];
    double dz[3] = {z[0] - v[0], z[1] - v[1], z[2] - v[2]};
    double cz = -dot3(h.n, wi);
    double seg = cz > 0.0 ? sqrt(dot3(dz, dz) / (pdf * cz)) : O_INF;
    double Lz[3];
    shade_radiance(sc, pr, pp, seed, pixel, frame, h.prim, z, h.n, v, foot_sum + seg, a0c, depth + 1, Lz);
    for (int a = 0; a < 3; ++a) L[a] += wgt * Lz[a];
}

void o_shade(const o_scene *sc, int32_t W, int32_t H, const double *gb, const o_probes *pr,
             const double *res, const double *resid, const o_params *pp, const int32_t *pix,
             int64_t npix, double *img, uint64_t seed, uint32_t frame)
{
    int64_t n = pix ? npix : (int64_t)W * H;
    O_PARALLEL
    for (int64_t q = 0; q < n; ++q) {
        int64_t p = pix ? pix[q] : q;
        const double *g = gb + GB_N * p;
        const double *r = res + R_N * p;
        double *o = img + 3 * p;
        for (int a = 0; a < 3; ++a) o[a] = g[GB_EMIT + a];
        if ((uint32_t)g[GB_PRIM] == O_MISS) continue;
        for (int a = 0; a < 3; ++a) o[a] += resid[3 * p + a];
        if (!(r[R_W] > 0.0)) continue;
        const double *x = g + GB_POS, *nx = g + GB_NRM, *rho = g + GB_ALB;
        double L[3], geo;
        if (res_is_sky(r)) {
            geo = dot3(nx, r + R_Y);
            if (geo <= 0.0) continue;
            if (!o_visible(sc, x, nx, r + R_Y, r + R_NY, 1)) continue;
            for (int a = 0; a < 3; ++a) L[a] = sc->sky[a];
        } else {
            const double *y = r + R_Y, *ny = r + R_NY;
            double v[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
            double d2 = dot3(v, v), d = sqrt(d2);
            double w[3] = {v[0] / d, v[1] / d, v[2] / d};
            double cx = dot3(nx, w), cy = -dot3(ny, w);
            if (cx <= 0.0 || cy <= 0.0) continue;
            geo = fmin(cx * cy / d2, pp->g_max);
            if (!o_visible(sc, x, nx, y, ny, 0)) continue;
            if (sc->glossy) {
                /* x_1 = x, x_2 = y: the first segment's density is the BSDF mixture's
                 * at x; a_0 = |x_0 - x_1|^2 / (4 pi cos) with x_0 the camera */
                double ks, ra, wo[3] = {pp->eye[0] - x[0], pp->eye[1] - x[1], pp->eye[2] - x[2]}, f[3];
                spec_of(sc, (uint32_t)g[GB_PRIM], &ks, &ra);
                double dc2 = dot3(wo, wo);
                normalize3(wo);
                double c1 = dot3(nx, wo);
                double a0c = c1 > 0.0 ? pp->foot_c * dc2 / (4.0 * O_PI * c1) : O_INF;
                double p1 = mix_pdf(rho, ks, ra, nx, wo, w);
                double foot = p1 > 0.0 ? sqrt(d2 / (p1 * cy)) : O_INF;
                shade_radiance(sc, pr, pp, seed, (uint32_t)p, frame, (uint32_t)r[R_PRIM], y, ny, x, foot, a0c, 1, L);
                bsdf(rho, ks, ra, nx, wo, w, f);
                for (int a = 0; a < 3; ++a) o[a] += f[a] * L[a] * geo * r[R_W];
                continue;
            }
            radiance_toward(sc, pr, (uint32_t)r[R_PRIM], y, ny, x, L);
        }
        if (sc->glossy) {
            double ks, ra, wo[3] = {pp->eye[0] - x[0], pp->eye[1] - x[1], pp->eye[2] - x[2]}, f[3];
            spec_of(sc, (uint32_t)g[GB_PRIM], &ks, &ra);
            normalize3(wo);
            bsdf(rho, ks, ra, nx, wo, r + R_Y, f);
            for (int a = 0; a < 3; ++a) o[a] += f[a] * L[a] * geo * r[R_W];
            continue;
        }
        for (int a = 0; a < 3; ++a) o[a] += rho[a] / O_PI * L[a] * geo * r[R_W];
    }
}

/* ---------------------------------------------------------------------------
 * Brute-force reference of what one pixel's estimate converges to:
 * L_e(x) + integral over the hemisphere of rho_x/pi * L(y; x) cos(theta_x),
 * by plain Monte Carlo with uniform hemisphere directions (a uniform sphere
 * direction mirrored into n_x's hemisphere, pdf 1/(2 pi)).  No resampling,
 * no bounding: a check of the whole resampled estimator (Eq. 9 is unbiased
 * for this integral).  Random stream: counter (sample, pixel, 99, 0).
 * ------------------------------------------------------------------------- */
void o_brute_force(const o_scene *sc, const o_probes *pr, const double *gb, int32_t W, int32_t H,
                   const int32_t *pix, int64_t npix, int64_t nsamples, uint64_t seed, double *out)
{
    O_PARALLEL
    for (int64_t q = 0; q < npix; ++q) {
        int64_t p = pix[q];
        const double *g = gb + GB_N * p;
        double *o = out + 3 * q;
        for (int a = 0; a < 3; ++a) o[a] = g[GB_EMIT + a];
        if (!pixel_active(sc, g)) continue;
        const double *x = g + GB_POS, *nx = g + GB_NRM, *rho = g + GB_ALB;
        double org[3], acc[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) org[a] = x[a] + sc->eps * nx[a];
        for (int64_t s = 0; s < nsamples; ++s) {
            double u[4], w[3], L[3];
            rand4(seed, (uint32_t)s, (uint32_t)p, 99u, 0u, u);
            o_sphere_dir(u[0], u[1], w);
            double c = dot3(nx, w);
            if (c < 0.0) { w[0] = -w[0]; w[1] = -w[1]; w[2] = -w[2]; c = -c; }
            o_hit h;
            if (closest_hit(sc, org, w, O_INF, &h)) {
                double y[3];
                for (int a = 0; a < 3; ++a) y[a] = org[a] + h.t * w[a];
                if (-dot3(h.n, w) <= 0.0) continue;
                radiance_toward(sc, pr, h.prim, y, h.n, x, L);
            } else {
                for (int a = 0; a < 3; ++a) L[a] = sc->sky[a];
            }
            for (int a = 0; a < 3; ++a) acc[a] += 2.0 * rho[a] * L[a] * c;
        }
        for (int a = 0; a < 3; ++a) o[a] += acc[a] / (double)nsamples;
    }
}

/* ---------------------------------------------------------------------------
 * Reference path tracer: the converged images the estimators are scored
 * against (the paper's evaluation compares with an unbiased path tracer,
 * Sec. 4).  A path starts at the pixel's primary vertex x (G-buffer) with
 * L = L_e(x).  Bounce b = 1, 2, ...: leaving a surface of albedo rho, a
 * cosine-distributed direction about its normal multiplies the throughput by
 * rho (the Lambertian BSDF times the cosine over the density); from bounce 4
 * on the path survives with probability P = min(1, max throughput component)
 * and its throughput is divided by P (Russian roulette); the ray from the
 * surface (offset eps along the normal) adds throughput x L_e of what it hits,
 * or throughput x sky on a miss, which ends the path; a surface of zero
 * albedo ends it too; at most 32 bounces.  Sample s, bounce b draws from
 * counter (pixel, s, 13, b): u0, u1 for the direction, u2 for the roulette.
 * out[q] = mean over samples s0 .. s0+spp-1.
 * ------------------------------------------------------------------------- */
void o_path_trace(const o_scene *sc, const double *gb, const int32_t *pix, int64_t npix, int32_t spp,
                  uint32_t s0, uint64_t seed, const double *eye, double *out)
{
    O_PARALLEL
    for (int64_t q = 0; q < npix; ++q) {
        const int64_t p = pix[q];
        const double *g = gb + GB_N * p;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int32_t s = 0; s < spp; ++s) {
            double x[3], n[3], rho[3], L[3], thr[3] = {1.0, 1.0, 1.0};
            for (int a = 0; a < 3; ++a) {
                x[a] = g[GB_POS + a];
                n[a] = g[GB_NRM + a];
                rho[a] = g[GB_ALB + a];
                L[a] = g[GB_EMIT + a];
            }
            if (sc->glossy) {
                /* glossy scene: at every vertex the BSDF mixture of the initial pass
                 * (glossy lobe with probability p_gloss, chosen by u3), throughput
                 * times f cos / pdf; roulette as below, after that product */
                uint32_t prim = (uint32_t)g[GB_PRIM];
                double wo[3] = {eye[0] - x[0], eye[1] - x[1], eye[2] - x[2]};
                normalize3(wo);
                for (uint32_t b = 1; b <= 32; ++b) {
                    double ks, ra;
                    spec_of(sc, prim, &ks, &ra);
                    if (rho[0] == 0.0 && rho[1] == 0.0 && rho[2] == 0.0 && !(ks > 0.0)) break;
                    double u[4], w[3], o[3], f[3];
                    rand4(seed, (uint32_t)p, s0 + (uint32_t)s, 13u, b, u);
                    double pg = p_gloss(rho, ks);
                    if (pg > 0.0 && u[3] < pg) {
                        if (!ggx_sample(n, wo, ra, u[0], u[1], w)) break;
                    } else {
                        o_cosine_dir(n, u[0], u[1], w);
                    }
                    double pd = mix_pdf(rho, ks, ra, n, wo, w);
                    if (!(pd > 0.0)) break;
                    bsdf(rho, ks, ra, n, wo, w, f);
                    double c = dot3(n, w);
                    for (int a = 0; a < 3; ++a) thr[a] *= f[a] * c / pd;
                    if (b >= 4) {
                        double P = fmin(1.0, fmax(thr[0], fmax(thr[1], thr[2])));
                        if (!(u[2] < P)) break;
                        for (int a = 0; a < 3; ++a) thr[a] /= P;
                    }
                    for (int a = 0; a < 3; ++a) o[a] = x[a] + sc->eps * n[a];
                    o_hit h;
                    if (!closest_hit(sc, o, w, O_INF, &h)) {
                        for (int a = 0; a < 3; ++a) L[a] += thr[a] * sc->sky[a];
                        break;
                    }
                    double emit[3];
                    for (int a = 0; a < 3; ++a) {
                        x[a] = o[a] + h.t * w[a];
                        n[a] = h.n[a];
                        wo[a] = -w[a];
                    }
                    prim = h.prim;
                    material(sc, h.prim, rho, emit);
                    for (int a = 0; a < 3; ++a) L[a] += thr[a] * emit[a];
                }
                for (int a = 0; a < 3; ++a) acc[a] += L[a];
                continue;
            }
            for (uint32_t b = 1; b <= 32; ++b) {
                if (rho[0] == 0.0 && rho[1] == 0.0 && rho[2] == 0.0) break;
                double u[4];
                rand4(seed, (uint32_t)p, s0 + (uint32_t)s, 13u, b, u);
                for (int a = 0; a < 3; ++a) thr[a] *= rho[a];
                if (b >= 4) {
                    double P = fmin(1.0, fmax(thr[0], fmax(thr[1], thr[2])));
                    if (!(u[2] < P)) break;
                    for (int a = 0; a < 3; ++a) thr[a] /= P;
                }
                double w[3], o[3];
                o_cosine_dir(n, u[0], u[1], w);
                for (int a = 0; a < 3; ++a) o[a] = x[a] + sc->eps * n[a];
                o_hit h;
                if (!closest_hit(sc, o, w, O_INF, &h)) {
                    for (int a = 0; a < 3; ++a) L[a] += thr[a] * sc->sky[a];
                    break;
                }
                double emit[3];
                for (int a = 0; a < 3; ++a) {
                    x[a] = o[a] + h.t * w[a];
                    n[a] = h.n[a];
                }
                material(sc, h.prim, rho, emit);
                for (int a = 0; a < 3; ++a) L[a] += thr[a] * emit[a];
            }
            for (int a = 0; a < 3; ++a) acc[a] += L[a];
        }
        for (int a = 0; a < 3; ++a) out[3 * q + a] = acc[a] / (double)spp;
    }
}

/* ---------------------------------------------------------------------------
 * Training samples of the learned cache (the MLP that can stand in for the
 * probe query; caches are interchangeable, Sec. 2 and Sec. 5).  The cache is
 * queried at the initial pass's candidates, so it is trained on them: sample
 * j (counter (j, frame, 10, 0)) takes pixel p = floor(u0 W H) and candidate
 * i = floor(u1 M) of that pixel, regenerated from the initial pass's own
 * counter (p, frame, 0, i) (direction u0, u1 about n_x from x + eps n_x).
 * Candidates that miss, land on a zero-albedo surface (where the cache is
 * never used) or belong to a pixel without a surface are invalid (all zero).
 * The label at the candidate y is a one-sample estimate of E(y, n_y)/pi: the
 * radiance arriving along a cosine-distributed direction (u2, u3) about n_y
 * from y + eps n_y, L_e(z) + rho_z Q(z_b, n_z) at the hit z with z_b biased
 * toward y (a gather past the probes, Sec. 3.2), or the sky.  qprobe receives
 * Q(y_b, n_y) with y_b biased toward x, the probe value the cache replaces.
 * (Selected reservoir samples would not do as training inputs: selection
 * follows the target, which contains the cache, so a region the cache
 * predicts dark would never be selected and never corrected.)
 * ------------------------------------------------------------------------- */
void o_mlp_batch(const o_scene *sc, const o_probes *pr, int32_t W, int32_t H, const double *gb, int32_t M,
                 int64_t B, uint64_t seed, uint32_t frame, double *pos, double *nrm, double *target,
                 int32_t *valid, double *qprobe)
{
    for (int64_t j = 0; j < B; ++j) {
        double u[4], c[4];
        rand4(seed, (uint32_t)j, frame, 10u, 0u, u);
        int64_t p = (int64_t)floor(u[0] * (double)W * (double)H);
        uint32_t i = (uint32_t)floor(u[1] * (double)M);
        const double *g = gb + GB_N * p;
        valid[j] = 0;
        for (int a = 0; a < 3; ++a) {
            pos[3 * j + a] = 0.0; nrm[3 * j + a] = 0.0; target[3 * j + a] = 0.0; qprobe[3 * j + a] = 0.0;
        }
        if (!pixel_active(sc, g)) continue;
        const double *x = g + GB_POS, *nx = g + GB_NRM;
        /* the candidate */
        double w[3], o[3];
        rand4(seed, (uint32_t)p, frame, 0u, i, c);
        o_cosine_dir(nx, c[0], c[1], w);
        for (int a = 0; a < 3; ++a) o[a] = x[a] + sc->eps * nx[a];
        o_hit hy;
        if (!closest_hit(sc, o, w, O_INF, &hy)) continue;
        double y[3], ny[3], alb[3], emit[3];
        for (int a = 0; a < 3; ++a) {
            y[a] = o[a] + hy.t * w[a];
            ny[a] = hy.n[a];
        }
        material(sc, hy.prim, alb, emit);
        if (alb[0] == 0.0 && alb[1] == 0.0 && alb[2] == 0.0) continue;
        /* its label */
        double wl[3], ol[3], L[3];
        o_cosine_dir(ny, u[2], u[3], wl);
        for (int a = 0; a < 3; ++a) ol[a] = y[a] + sc->eps * ny[a];
        o_hit h;
        if (closest_hit(sc, ol, wl, O_INF, &h)) {
            double z[3];
            for (int a = 0; a < 3; ++a) z[a] = ol[a] + h.t * wl[a];
            radiance_toward_ex(sc, pr, h.prim, z, h.n, y, 0, NULL, L);
        } else {
            for (int a = 0; a < 3; ++a) L[a] = sc->sky[a];
        }
        /* the probe value the cache replaces at y, biased toward x */
        double yb[3], q[3];
        o_view_bias(y, x, pr->bias_dist, yb);
        probe_query(pr, yb, ny, 0, q);
        valid[j] = 1;
        for (int a = 0; a < 3; ++a) {
            pos[3 * j + a] = y[a]; nrm[3 * j + a] = ny[a]; target[3 * j + a] = L[a]; qprobe[3 * j + a] = q[a];
        }
    }
}
