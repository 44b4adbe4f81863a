/*
 * gi.h - C ABI of the MI355X DDGI-resampling library (libgi.so).
 *
 * Per-pixel hot path of "Dynamic Diffuse Global Illumination Resampling"
 * (Majercik, Mueller, Keller, Nowrouzezahrai, McGuire, EGSR 2021):
 * candidate generation, a target built from DDGI probe irradiance, streaming
 * weighted-reservoir resampling, temporal and spatial reuse with visibility
 * rays, and shading, for an analytic scene (room + spheres + boxes).
 *
 * Conventions shared by every entry point
 *  - Every buffer pointer is DEVICE memory owned by the caller.  The library
 *    allocates nothing, keeps no pointer after a call returns, and has no
 *    mutable global state; buffers must stay valid until the stream's work
 *    has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call is asynchronous on that stream.
 *  - Arguments are validated on the host before anything is launched; a
 *    failed validation returns an error status and launches nothing.
 *    GI_ERR_LAUNCH reports a failed launch; device faults surface at the
 *    caller's next synchronisation.
 *  - Pixel p = j*width + i, row 0 at the top.  Image planes are SoA arrays of
 *    float4 (16-byte records), one record per pixel.
 *  - Identical inputs, seed and frame give bit-identical outputs.
 *  - All arithmetic is FP32.  Random numbers come from Philox4x32-10 keyed
 *    by (seed) with counter (pixel or probe, frame, pass, block).
 */
#ifndef GI_H
#define GI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gi_status {
    GI_OK = 0,
    GI_ERR_NULL = 1,      /* a required pointer is NULL */
    GI_ERR_SHAPE = 2,     /* sizes disagree or exceed a limit */
    GI_ERR_PARAM = 3,     /* a parameter is out of its documented range */
    GI_ERR_ALIAS = 4,     /* an output buffer aliases an input buffer */
    GI_ERR_LAUNCH = 5,    /* the kernel launch failed (hipGetLastError) */
    GI_ERR_DEVICE = 6     /* no usable HIP device */
} gi_status;

#define GI_MISS 0xFFFFFFFFu          /* primitive id of "no hit" / sky */
#define GI_EMPTY_TAG 0xFFFFFFFFu     /* tag of a reservoir that holds no sample */
#define GI_MAX_M 32u                 /* largest candidate count per pixel */
#define GI_MAX_K 8u                  /* largest spatial neighbour count */
#define GI_MAX_PROBE_RAYS 1024u      /* largest probe-update ray count */

/* Primitive record, 64 bytes.  type 0 = sphere (size[0] = radius),
 * type 1 = axis-aligned box (size = half extents). */
typedef struct gi_prim {
    float center[3];
    uint32_t type;
    float size[3];
    float pad0;
    float albedo[3];     /* diffuse albedo rho */
    float pad1;
    float emit[3];       /* emitted radiance L_e */
    float pad2;
} gi_prim;

/* Analytic scene.  The room (if has_room) is the inside of the box
 * [room_lo, room_hi]; its six walls take primitive ids n_prims + 2*axis + side
 * (side 1 = the room_hi wall).  Rays that leave an open scene see `sky`.
 * Optional uniform-grid accelerator over [grid_lo, grid_hi] with grid_res
 * cells (x fastest): cell c lists primitive ids cell_items[cell_start[c] ..
 * cell_start[c+1]); build it with gi_accel_build_host.  cell_start == NULL
 * selects brute force over all primitives.  Results never depend on it. */
typedef struct gi_scene {
    const gi_prim *prims;
    uint32_t n_prims;
    uint32_t has_room;
    float room_lo[3], room_hi[3];
    float wall_albedo[3], wall_emit[3];
    float sky[3];
    float eps;                       /* ray origins are lifted by eps along the normal */
    uint32_t grid_res[3];
    float grid_lo[3], grid_hi[3];
    const uint32_t *cell_start;      /* grid_res[0]*grid_res[1]*grid_res[2] + 1 entries */
    const uint32_t *cell_items;
    uint32_t n_items;                /* entries of cell_items (= cell_start[last]) */
    uint32_t options;                /* GI_OPT_* bits */
} gi_scene;

#define GI_OPT_NO_LDS 1u             /* trace from global memory even when the scene fits LDS */

/* Pinhole camera: the ray through pixel (i, j) has direction
 * normalize(fwd + sx*right + sy*up), sx = (2(i+.5)/W - 1) tan_half_fovy W/H,
 * sy = (1 - 2(j+.5)/H) tan_half_fovy. */
typedef struct gi_camera {
    float eye[3], fwd[3], right[3], up[3];
    float tan_half_fovy;
    uint32_t width, height;
} gi_camera;

/* G-buffer of primary vertices, four float4 planes of width*height records:
 *   pos_depth = (x, y, z, view depth), nrm_prim = (n_x, n_y, n_z, prim id as
 *   uint32 bits), albedo = (r, g, b, 0), emit = (r, g, b, 0).
 * A pixel whose primary ray leaves the scene has prim = GI_MISS and emit = sky. */
typedef struct gi_gbuffer {
    uint32_t width, height;
    float *pos_depth;
    float *nrm_prim;
    float *albedo;
    float *emit;
} gi_gbuffer;

/* DDGI probe volume.  Probe (i, j, k), index i + dims[0]*(j + dims[1]*k),
 * sits at lo + (idx + 0.5) * spacing.  Each probe owns an octahedral
 * irradiance tile (irr_res^2 texels of E/pi, RGB) and depth tile (dep_res^2
 * texels of the mean and mean square hit distance), each with a one-texel
 * gutter that mirrors the interior along the tile edge (corners take the
 * diagonally opposite interior texel).  They are stored as bilinear quads:
 *   irr: per probe (irr_res+1)^2 records of 12 floats; record cy*(irr_res+1)+cx
 *        holds the RGB of padded texels (cx,cy), (cx+1,cy), (cx,cy+1),
 *        (cx+1,cy+1) in that order (3888 bytes per probe);
 *   dep: per probe (dep_res+1)^2 records of 8 floats, (mean, mean^2) of the
 *        same four padded texels (9248 bytes per probe).
 * irr_res must be 8 and dep_res 16.  bias_dist is the view-path bias d,
 * var_floor the Chebyshev variance floor, d_max the probe-ray depth clamp. */
typedef struct gi_probes {
    uint32_t dims[3];
    uint32_t irr_res, dep_res;
    float lo[3], spacing[3];
    float bias_dist, var_floor, d_max;
    float *irr;
    float *dep;
} gi_probes;

/* Reservoirs, SoA planes of width*height records:
 *   y_W      float4 (y.x, y.y, y.z, W)        W = contribution weight
 *   n_wsum   float4 (n_y.x, n_y.y, n_y.z, wsum)
 *   L_M      float4 (L.r, L.g, L.b, M as uint32 bits)   L = cached radiance of y
 *   tag_prim uint2  (tag, primitive id of y)
 * A sample that left an open scene stores its direction in y and n_y = 0.
 * tag = origin pixel << 9 | candidate << 4 | (frame & 15); GI_EMPTY_TAG = none. */
typedef struct gi_reservoirs {
    uint32_t width, height;
    float *y_W;
    float *n_wsum;
    float *L_M;
    uint32_t *tag_prim;
} gi_reservoirs;

/* Resampling parameters. */
typedef struct gi_params {
    uint32_t M;          /* candidates per pixel, 1..GI_MAX_M */
    uint32_t k;          /* spatial neighbours, 0..GI_MAX_K */
    float radius;        /* spatial disk radius in pixels, >= 0 */
    float g_max;         /* geometry-term bound G_max (Sec. 3.5), > 0 */
    float cos_n;         /* reuse normal threshold (cosine) */
    float depth_rel;     /* reuse relative depth threshold */
    float m_cap;         /* temporal history cap, multiple of the current M */
    uint32_t unbiased;   /* 1: visibility-tested 1/Z normalisation, 0: 1/M */
} gi_params;

/* Probe-update parameters. */
typedef struct gi_probe_params {
    uint32_t rays;       /* rays per probe, 1..GI_MAX_PROBE_RAYS */
    float hysteresis;    /* stored = h*old + (1-h)*new, in [0, 1] */
    float sharpness;     /* exponent of the depth-moment cosine lobe, > 0 */
} gi_probe_params;

/* Human-readable name of a status code (static storage). */
const char *gi_status_string(gi_status s);

/* Number of the HIP device the calling thread uses, or -1 (host query). */
int gi_device(void);

/* Primary vertices (Sec. 3.1: the primary vertex x, with L_e(x) of Eq. 9):
 * one pinhole ray per pixel centre, closest hit, written to `out`.
 * out->width/height must equal the camera's. */
gi_status gi_trace_gbuffer(const gi_scene *scene, const gi_camera *cam, gi_gbuffer *out,
                           void *stream);

/* Augmented probe update E_DDGI+ (Eq. 5, Sec. 3.2): every probe traces
 * `rays` uniform-sphere rays (counter (probe, frame, 9, ray)); a hit h brings
 * L_e(h) + rho_h * Q_in(h_b, n_h) with h_b moved toward the probe by
 * min(bias_dist, t/2), a miss brings the sky; irradiance texels take the
 * cosine-weighted mean, depth texels the cos^sharpness-weighted mean of
 * (d, d^2) with d = min(t, d_max); stored = h*in + (1-h)*new; gutters filled.
 * Reads only `in`, writes only `out` (same layout, must not alias). */
gi_status gi_probe_update(const gi_scene *scene, const gi_probes *in, gi_probes *out,
                          const gi_probe_params *pp, uint64_t seed, uint32_t frame, void *stream);

/* Probe query Q(p, n) = E(p, n)/pi (Eq. 4; probe weights of the DDGI volume
 * the paper builds on, with the probes' mean visibility of Sec. 3.2):
 * trilinear x backface x Chebyshev-visibility blend of the 8 probes of p's
 * cell, normalised.  p, nrm: n points as 3 floats each; out: 3 floats each. */
gi_status gi_probe_query(const gi_probes *probes, uint32_t n, const float *p, const float *nrm,
                         float *out, void *stream);

/* Initial resampling (Sec. 3.1 steps 1-2, Fig. 2, Sec. 3.5, Sec. 3.6): per
 * pixel, M cosine-sampled candidates y_i (counter (pixel, frame, 0, i)), each
 * traced, its radiance L(y_i) = L_e + rho Q(view-path-biased y_i, n_y)
 * evaluated, weighted w = p_hat/p_A with p_hat = lum(rho_x/pi L) min(G, g_max)
 * and streamed through a weighted reservoir (replace iff u*wsum < w); W =
 * wsum/(M p_hat(y)).  resid (float4 plane, rgb used) receives the residual
 * transport rho_x L(y_0) max(0, 1 - g_max/G_0) of candidate 0 (Eq. 9).
 * Pixels that miss or have zero albedo get an empty reservoir with M = 0. */
gi_status gi_resample_initial(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes,
                              const gi_params *params, gi_reservoirs *out, float *resid,
                              uint64_t seed, uint32_t frame, void *stream);

/* Temporal reuse (Sec. 3.1 step 2, Sec. 3.6): x is projected with prev_cam;
 * if the previous pixel is a hit with n.n_prev >= cos_n and |depth -
 * depth_prev| <= depth_rel*depth, the history reservoir (M capped at
 * m_cap*M) is merged after the pixel's own, with weights p_hat_x(y)W M using
 * the cached L.  Unbiased mode: Z counts the domains whose target supports y
 * and that see y (one visibility ray each, the history domain from its
 * previous-frame vertex); a sample x cannot see is dropped.
 * cur/prev G-buffers and all reservoir sets must share one size; `out` must
 * not alias `cur_in` or `history`. */
gi_status gi_resample_temporal(const gi_scene *scene, const gi_gbuffer *gb, const gi_gbuffer *gb_prev,
                               const gi_camera *prev_cam, const gi_reservoirs *cur_in,
                               const gi_reservoirs *history, const gi_params *params,
                               gi_reservoirs *out, uint64_t seed, uint32_t frame, void *stream);

/* Spatial reuse, pass `pass` (Sec. 3.1 step 2, Sec. 3.6): merge the pixel's
 * own reservoir, then k neighbours drawn uniformly in the disk of `radius`
 * pixels (counter (pixel, frame, 2+pass, j)) that pass the normal/depth test;
 * normalisation as in gi_resample_temporal.  `out` must not alias `in`. */
gi_status gi_resample_spatial(const gi_scene *scene, const gi_gbuffer *gb, const gi_reservoirs *in,
                              const gi_params *params, uint32_t pass, gi_reservoirs *out,
                              uint64_t seed, uint32_t frame, void *stream);

/* Shading (Sec. 3.1 steps 3-4, Eq. 9): L_o = L_e(x) + resid(x) +
 * rho_x/pi L(y; x) min(G, g_max) V(x, y) W with a fresh radiance query biased
 * toward this x and one shadow ray.  out_rgba: float4 plane (rgb, 1). */
gi_status gi_shade(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes,
                   const gi_reservoirs *res, const float *resid, const gi_params *params,
                   float *out_rgba, void *stream);

/* Host-side builder of the optional uniform-grid accelerator.  prims: HOST
 * array of n records.  Cells cover [lo, hi] with res cells per axis; a
 * primitive is listed in every cell its bounding box (padded by 1e-3 cell)
 * overlaps, in increasing id order.  cell_start (host, ncells+1) is always
 * written; items (host, `capacity` entries) is written when large enough.
 * *n_items receives the required count; GI_ERR_SHAPE if capacity is short. */
gi_status gi_accel_build_host(const gi_prim *prims, uint32_t n, const float lo[3], const float hi[3],
                              const uint32_t res[3], uint32_t *cell_start, uint32_t *items,
                              uint32_t capacity, uint32_t *n_items);

/* Philox4x32-10 blocks on the device (test hook for bit-exact RNG parity):
 * ctr: n counters of 4 uint32, out: n blocks of 4 uint32. */
gi_status gi_philox(uint64_t seed, uint32_t n, const uint32_t *ctr, uint32_t *out, void *stream);

/* Closest hit of n rays (test hook for the tracer): org, dir: 3 floats each
 * (dir unit length); out: 4 floats per ray (t, n_x, n_y, n_z), prim: id or
 * GI_MISS (t = +inf on a miss). */
gi_status gi_trace_rays(const gi_scene *scene, uint32_t n, const float *org, const float *dir,
                        float *out, uint32_t *prim, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GI_H */
