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
 *    mutable global state besides the per-GPU scratch of
 *    gi_mlp_train_step_noalloc; buffers must stay valid until the stream's
 *    work has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call is asynchronous on that stream.
 *  - Arguments are validated on the host before anything is launched; a
 *    failed validation returns an error status and launches nothing.
 *  - An empty image (width or height 0) or an empty batch (n = 0) passes the
 *    same checks and then returns GI_OK without launching anything (except
 *    gi_mlp_grad / gi_mlp_train_step, which still write the zero gradient of
 *    an empty batch).
 *    GI_ERR_LAUNCH reports a failed launch; device faults surface at the
 *    caller's next synchronisation.
 *  - Pixel p = j*width + i, row 0 at the top.  Image planes are SoA arrays of
 *    float4 (16-byte records), one record per pixel.
 *  - Identical inputs, seed and frame give bit-identical outputs.
 *  - All arithmetic is FP32.  Random numbers come from Philox4x32-10 keyed
 *    by (seed) with counter (pixel or probe, frame, pass, block).
 *  - Against a single-entry-point design with optional arguments, the
 *    learned cache has its own entry points (gi_resample_initial_mlp,
 *    gi_shade_mlp) with a caller workspace, the probe update reads one
 *    volume and writes another (each probe reads its neighbours' previous
 *    textures), shading takes seed and frame (the glossy recursion samples),
 *    and precisions are chosen per buffer (G-buffer format, cache precision)
 *    rather than by a general dtype argument.
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
 * type 1 = axis-aligned box (size = half extents).  spec and rough describe
 * an optional glossy layer (Sec. 3.3): f = albedo/pi + spec * D G1 G1 /
 * (4 cos_o cos_i) with isotropic GGX D of roughness `rough` and separable
 * Smith masking; they are read only in scenes with GI_OPT_GLOSSY. */
typedef struct gi_prim {
    float center[3];
    uint32_t type;
    float size[3];
    float pad0;
    float albedo[3];     /* diffuse albedo rho */
    float spec;          /* weight k_s of the GGX layer, 0 = Lambertian */
    float emit[3];       /* emitted radiance L_e */
    float rough;         /* GGX roughness alpha in (0, 1] (with spec > 0) */
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
    uint32_t n_emitters;             /* emissive spheres light sampling draws from, <= GI_MAX_EMITTERS */
    uint32_t emitters[32];           /* their primitive ids (each a sphere with emission) */
} gi_scene;

#define GI_MAX_EMITTERS 32u

#define GI_OPT_NO_LDS 1u             /* trace from global memory even when the scene fits LDS */
#define GI_OPT_GLOSSY 2u             /* primitives may carry a glossy layer (gi_prim spec, rough): the
                                        kernels with the glossy BSDF, glossy L_DDGI+ (Eq. 6) and the
                                        shading recursion (Eq. 7-8) run; without it spec is ignored */

/* Pinhole camera: the ray through pixel (i, j) has direction
 * normalize(fwd + sx*right + sy*up), sx = (2(i+.5)/W - 1) tan_half_fovy W/H,
 * sy = (1 - 2(j+.5)/H) tan_half_fovy. */
typedef struct gi_camera {
    float eye[3], fwd[3], right[3], up[3];
    float tan_half_fovy;
    uint32_t width, height;
} gi_camera;

/* G-buffer of primary vertices, four planes of width*height records.
 * format GI_GB_F32: four float4 planes, pos_depth = (x, y, z, view depth),
 *   nrm_prim = (n_x, n_y, n_z, prim id as uint32 bits), albedo = (r, g, b, 0),
 *   emit = (r, g, b, 0).
 * format GI_GB_F16 (normals and albedo in half precision, rounded to nearest
 *   even): nrm_prim holds 8-byte records (half n_x, n_y, n_z; uint16 prim id,
 *   0xFFFF = miss), albedo 8-byte records (half r, g, b, 0); pos_depth and
 *   emit stay float4; readers renormalise the half-precision normal.  Scenes
 *   must have fewer than 65535 - 6 primitives.
 * A pixel whose primary ray leaves the scene has prim = GI_MISS and emit = sky. */
typedef struct gi_gbuffer {
    uint32_t width, height;
    float *pos_depth;
    float *nrm_prim;
    float *albedo;
    float *emit;
    uint32_t format;     /* GI_GB_F32 or GI_GB_F16 */
    uint32_t pad;
    float eye[3];        /* camera position the buffer was traced from (view direction of glossy
                            primary vertices); gi_trace_gbuffer does not write it, the caller sets it */
    float pad2;
} gi_gbuffer;

#define GI_GB_F32 0u
#define GI_GB_F16 1u

/* Texel formats of a probe volume (gi_probes.texel) */
#define GI_TEXEL_F32 0u   /* FP32 texels */
#define GI_TEXEL_F16 1u   /* IEEE binary16 texels */

/* DDGI probe volume.  Probe (i, j, k), index i + dims[0]*(j + dims[1]*k),
 * sits at lo + (idx + 0.5) * spacing.  Each probe owns an octahedral
 * irradiance tile (irr_res^2 texels of E/pi, RGB) and depth tile (dep_res^2
 * texels of the mean and mean square hit distance), each with a one-texel
 * gutter that mirrors the interior along the tile edge (corners take the
 * diagonally opposite interior texel).  Texels are stored in the volume's
 * texel format:
 *   GI_TEXEL_F32: FP32 values, depth texels as (mean, mean square);
 *   GI_TEXEL_F16: IEEE binary16 values (gi_probe_update rounds to nearest
 *        even), depth texels as (mean, variance), the variance being the mean
 *        square minus the squared mean (the query rebuilds the mean square as
 *        variance + mean^2).
 * They are stored as bilinear quads:
 *   irr: (irr_res+1)^2 records of 12 values per probe (48 bytes in FP32, 24
 *        in binary16), quad-major: record q = cy*(irr_res+1)+cx of probe i is
 *        record q*P + i (P probes), and holds the RGB of padded texels
 *        (cx,cy), (cx+1,cy), (cx,cy+1), (cx+1,cy+1) in that order (3888 or
 *        1944 bytes per probe in all);
 *   dep: per probe (dep_res+1)^2 records of 8 values (32 or 16 bytes), the
 *        two depth values of the same four padded texels, probe-major (9248
 *        or 4624 bytes per probe).
 * irr_res must be 8 and dep_res 16; the volume holds at most 464,000
 * probes (each texture then stays under 4 GiB, so kernels address it with
 * 32-bit byte offsets; larger volumes return GI_ERR_SHAPE); texel must be
 * one of the formats above (else GI_ERR_PARAM).  bias_dist is the view-path
 * bias d, var_floor the Chebyshev variance floor, d_max the probe-ray depth
 * clamp. */
typedef struct gi_probes {
    uint32_t dims[3];
    uint32_t irr_res, dep_res;
    float lo[3], spacing[3];
    float bias_dist, var_floor, d_max;
    uint32_t texel;       /* GI_TEXEL_F32 or GI_TEXEL_F16 */
    void *irr;            /* device, records as above */
    void *dep;            /* device, records as above */
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
    float m_cap;         /* temporal history cap: the history's M is capped at
                            floor(m_cap * (M + M_light)), computed in double */
    uint32_t unbiased;   /* 1: visibility-tested 1/Z normalisation, 0: 1/M */
    uint32_t M_light;    /* emitter-sampled candidates per pixel; M + M_light <= GI_MAX_M */
    uint32_t subsample;  /* n >= 1: pixel (x, y) draws candidates in frame f iff (x + y + f) % n == 0 */
    float foot_c;        /* glossy scenes: footprint threshold c of the shading recursion (Eq. 8), >= 0 */
    uint32_t glossy_depth; /* glossy scenes: most glossy vertices the recursion visits, 1..GI_MAX_GLOSSY_DEPTH */
} gi_params;

#define GI_MAX_GLOSSY_DEPTH 16u

/* Probe-update parameters. */
typedef struct gi_probe_params {
    uint32_t rays;       /* rays per probe, 1..GI_MAX_PROBE_RAYS */
    float hysteresis;    /* stored = h*old + (1-h)*new, in [0, 1] */
    float sharpness;     /* exponent of the depth-moment cosine lobe, > 0 */
    float distance_slider; /* >= 0; 0 switches the emission distance heuristic off */
} gi_probe_params;

/* Human-readable name of a status code (static storage). */
const char *gi_status_string(gi_status s);

/* Number of the HIP device the calling thread uses, or -1 (host query). */
int gi_device(void);

/* Hash of the sources and compiler flags this library was built from (16
 * hex digits, static storage): build provenance, compared by the loader with
 * the sources it ships with. */
const char *gi_build_hash(void);

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
 * With distance_slider s > 0 (the distance heuristic of Sec. 3.2) emission
 * reached at ray length t is scaled by (t / (t + s d_b))^2, d_b = the
 * probe's own mean depth (input texture) in the backward direction, clipped
 * to the distance from the probe to its cell boundary along that direction.
 * The blend reads the old texels and stores the new ones in the volume's
 * texel format (binary16: each stored value rounded to nearest even).
 * Reads only `in`, writes only `out` (same layout and texel format, else
 * GI_ERR_SHAPE / GI_ERR_PARAM; must not alias). */
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
 * wsum/(M p_hat(y)).  With M_light > 0 (Sec. 3.1 step 1 samples the emitters
 * too), candidates i = M .. M+M_light-1 are points uniform in the area of an
 * emitter chosen uniformly from scene->emitters (u0 the emitter, u1, u2 the
 * point, u3 the decision); every candidate's weight is then p_hat over the
 * balance-heuristic mixture density (M p_A + M_light p_light)/(M + M_light)
 * and M + M_light candidates are counted.  With subsample n > 1 (the
 * subsampling of Sec. 6) only pixels with (x + y + frame) % n == 0 draw
 * candidates; the others get an empty reservoir (M = 0) and take their
 * samples from temporal reuse (the history cap does not depend on the
 * pixel's own M) and spatial reuse, but still estimate the residual
 * from candidate 0.  resid (float4 plane, rgb used)
 * receives the residual transport rho_x L(y_0) max(0, 1 - g_max/G_0) of
 * candidate 0 (Eq. 9).  Pixels that miss or have zero albedo get an empty
 * reservoir with M = 0.  Images of more than 2^23 pixels return GI_ERR_SHAPE
 * (a tag holds a 23-bit origin pixel). */
gi_status gi_resample_initial(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes,
                              const gi_params *params, gi_reservoirs *out, float *resid,
                              uint64_t seed, uint32_t frame, void *stream);

/* Temporal reuse (Sec. 3.1 step 2, Sec. 3.6): x is projected with prev_cam;
 * if the previous pixel is a hit with n.n_prev >= cos_n and |depth -
 * depth_prev| <= depth_rel*depth, the history reservoir (M capped at
 * floor(m_cap*(M + M_light)), the per-frame candidate count, so that a pixel
 * that drew no candidates this frame still takes over its history) is
 * merged after the pixel's own, with weights p_hat_x(y)W M using
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
 * toward this x and one shadow ray.  out_rgba: float4 plane (rgb, 1).
 * In a glossy scene f(x) replaces rho_x/pi and L(y; x) follows the specular
 * recursion (Sec. 3.3, Eq. 7-8): glossy vertices draw one lobe direction each
 * (counter (pixel, frame, 16, depth)) and trace it while the path footprint
 * stays below a_0 * foot_c, else read the probes; seed and frame drive it
 * (unused in Lambertian scenes). */
gi_status gi_shade(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes,
                   const gi_reservoirs *res, const float *resid, const gi_params *params,
                   float *out_rgba, uint64_t seed, uint32_t frame, void *stream);

/* ==========================================================================
 * Learned radiance cache (the paper treats the irradiance cache as
 * interchangeable: Sec. 2 and Sec. 5 name neural radiance caching as an
 * alternative).  A small MLP C(y, n) ~ E(y, n)/pi replaces the probe query in
 * the target; the probe query stays the fallback.
 *
 * Network: inputs y normalised to [0,1]^3 by [pos_lo, pos_hi] and the raw
 * normal n; each of the 6 values v is encoded as [v, sin(2^j pi v),
 * cos(2^j pi v), j = 0..5] (feature 13*i + e, 78 in all); layers 78 -> 64 ->
 * 64 -> 64 -> 64 -> 3, ReLU on the hidden layers, linear output (used as
 * max(0, C)).  Parameters (FP32 master copy, GI_MLP_N_PARAMS floats): W1
 * (64x78 row-major, out x in), b1, W2 (64x64), b2, W3, b3, W4, b4, W5 (3x64),
 * b5.
 *
 * Precision: BF16 inference rounds every GEMM operand (encoded input,
 * weights, hidden activations) to BF16, nearest even, and accumulates in
 * FP32 (biases FP32).  FP8 inference stores operands as OCP E4M3FN values
 * x/s, saturating at +-448, with power-of-two scales: per weight matrix the
 * smallest power of two s with amax|W_l| <= 448 s, per layer input the
 * activation scale of layer l (scales[5 + l]) rounded up to a power of two;
 * products accumulate in FP32 and are scaled back by s_w*s_a.  Training is BF16 (gradients that enter a
 * product are rounded to BF16 too) with FP32 master weights and Adam moments.
 * ========================================================================== */
#define GI_MLP_N_PARAMS 17731u
#define GI_MLP_WEIGHT_BYTES 40064u   /* 38 MFMA fragments x 64 lanes x 16 B + 288 FP32 biases */
#define GI_MLP_MAX_BATCH (1u << 20)  /* largest training batch per call */

typedef enum gi_mlp_precision { GI_MLP_BF16 = 0, GI_MLP_FP8 = 1 } gi_mlp_precision;

/* When the resampling entry points use the cache. */
typedef enum gi_mlp_mode {
    GI_MLP_AUTO = 0,     /* when state[GI_MLP_STATE_USABLE] != 0 (decided on the device) */
    GI_MLP_ALWAYS = 1,   /* always the cache */
    GI_MLP_NEVER = 2     /* always the probe query */
} gi_mlp_mode;

/* Words of gi_mlp.state (uint32; FP32 values stored as their bits). */
#define GI_MLP_STATE_USABLE 0     /* 1 when AUTO mode uses the cache */
#define GI_MLP_STATE_STEPS 1      /* Adam steps taken */
#define GI_MLP_STATE_NONFINITE 2  /* non-finite outputs in the last training batch */
#define GI_MLP_STATE_EMA_ERR 3    /* EMA of BATCH_ERR (float) */
#define GI_MLP_STATE_LOSS 4       /* loss of the last training batch (float) */
#define GI_MLP_STATE_VALID 5      /* valid samples in the last training batch */
#define GI_MLP_STATE_BATCH_ERR 6  /* cache / probe squared-error ratio of the last batch (float) */
#define GI_MLP_STATE_WORDS 16

typedef struct gi_mlp {
    float *params;        /* GI_MLP_N_PARAMS FP32 master parameters */
    float *adam_m;        /* GI_MLP_N_PARAMS Adam first moments (zero at start) */
    float *adam_v;        /* GI_MLP_N_PARAMS Adam second moments (zero at start) */
    float *ema;           /* GI_MLP_N_PARAMS exponential moving average of the parameters, or
                             NULL; when set (and after the first Adam step) inference uses the
                             bias-corrected average ema / (1 - ema_decay^t) */
    void *weights;        /* GI_MLP_WEIGHT_BYTES inference operands, written by gi_mlp_prepare */
    float *scales;        /* 16 floats: [0..4] FP8 weight scales (gi_mlp_prepare), [5..9] FP8
                             activation scales of the layer inputs (gi_mlp_grad or the caller) */
    uint32_t *state;      /* GI_MLP_STATE_WORDS words, zero at start */
    float pos_lo[3];      /* position normalisation box */
    float pos_hi[3];
    uint32_t precision;   /* gi_mlp_precision of inference */
    uint32_t mode;        /* gi_mlp_mode */
    uint32_t warmup_steps;/* AUTO: Adam steps before the cache may be used */
    float max_rel_err;    /* AUTO: largest EMA of the cache / probe squared-error ratio, > 0 (1: the
                             cache is used while it predicts the labels no worse than the probes) */
    float ema_decay;      /* decay of the parameter average, in [0, 1) */
    uint32_t pad;
} gi_mlp;

/* Initialise the master parameters: He-uniform weights, W[o][i] = (2u - 1)
 * sqrt(6 / fan_in) with u from counter (parameter index, 0, 12, 0) (first
 * word), zero biases; Adam moments, the parameter average and the state are
 * zeroed, then gi_mlp_prepare runs. */
gi_status gi_mlp_init(const gi_mlp *mlp, uint64_t seed, void *stream);

/* Convert the inference parameters (the bias-corrected average when `ema`
 * is set and state STEPS > 0, else the master parameters) into the inference
 * operands: BF16 or FP8 MFMA fragments per `precision` and FP32 biases; FP8
 * also writes the weight scales.  Must run after any change of params, ema
 * or precision, before inference. */
gi_status gi_mlp_prepare(const gi_mlp *mlp, void *stream);

/* Cache output C(y, n) for n points: pos4, nrm4 are float4 planes (xyz used),
 * out4 receives (C_r, C_g, C_b, 0).  Runs whatever the mode (the state is
 * not consulted). */
gi_status gi_mlp_infer(const gi_mlp *mlp, uint32_t n, const float *pos4, const float *nrm4, float *out4,
                       void *stream);

/* Training samples: the cache is queried at the initial pass's candidates,
 * so it is trained on them.  Sample j (counter (j, frame, 10, 0)) takes pixel
 * p = floor(u0 W H) and candidate i = floor(u1 M) of the initial pass
 * (counter (p, frame, 0, i), traced as gi_resample_initial traces it); its
 * label is the radiance arriving along a cosine-distributed direction (u2,
 * u3) about n_y, L_e(z) + rho_z Q(z_b, n_z) at the hit z with z_b biased
 * toward y (a one-bounce gather past the probes, Sec. 3.2), or the sky.
 * Outputs (float4 planes of n): pos4 (y, 0), nrm4 (n_y, 0), target4 (label,
 * valid 1/0), qprobe4 (Q(y_b, n_y) with y_b biased toward the pixel's x: the
 * probe value the cache replaces, 0).  A sample whose pixel has no surface,
 * whose candidate misses or lands on a zero-albedo surface is invalid (all
 * zero).  M in 1..GI_MAX_M (the initial pass's candidate count).
 * Glossy scenes (GI_OPT_GLOSSY) return GI_ERR_PARAM: the cache serves Lambertian
 * scenes. */
gi_status gi_mlp_make_batch(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes, uint32_t M,
                            uint32_t n, uint64_t seed, uint32_t frame, float *pos4, float *nrm4,
                            float *target4, float *qprobe4, void *stream);

/* Device workspace bytes gi_mlp_grad / gi_mlp_train_step need for n samples. */
uint64_t gi_mlp_train_workspace_bytes(uint32_t n);

/* Gradient of the relative-L2 loss, mean over valid samples and channels of
 * (C - t)^2 / (sg(C)^2 + 0.01), with BF16 operands as above; writes grad
 * (GI_MLP_N_PARAMS floats, caller-owned) and, into state, LOSS, VALID,
 * NONFINITE and BATCH_ERR = sum (max(0,C) - t)^2 / sum (q - t)^2 over valid
 * samples and channels: the squared error of the cache, as the target uses
 * it, against the batch's labels t relative to that of the probe query q
 * (qprobe4; NULL gives 0; a zero denominator gives FLT_MAX unless the
 * numerator is zero too); writes
 * the FP8 scale of every layer input, the smallest power of two s with
 * activation amax <= 448 s (1 when the amax is 0), into scales[5..9].  The sums
 * are reduced in a fixed order (deterministic). */
gi_status gi_mlp_grad(const gi_mlp *mlp, uint32_t n, const float *pos4, const float *nrm4,
                      const float *target4, const float *qprobe4, float *grad, void *workspace,
                      uint64_t workspace_bytes, void *stream);

/* One Adam step (beta 0.9, 0.99, eps 1e-8, bias-corrected with step t >= 1)
 * on the master parameters with gradient grad; when `ema` is set, ema =
 * ema_decay * ema + (1 - ema_decay) * params afterwards; then gi_mlp_prepare.  Updates
 * state: STEPS = t, EMA_ERR (0.9 old + 0.1 BATCH_ERR, or BATCH_ERR at t = 1)
 * and USABLE = (t >= warmup_steps && NONFINITE == 0 && EMA_ERR <=
 * max_rel_err && every parameter finite). */
gi_status gi_mlp_adam(const gi_mlp *mlp, const float *grad, uint32_t t, float lr, void *stream);

/* gi_mlp_grad followed by gi_mlp_adam, the gradient kept in the workspace. */
gi_status gi_mlp_train_step(const gi_mlp *mlp, uint32_t n, const float *pos4, const float *nrm4,
                            const float *target4, const float *qprobe4, uint32_t t, float lr,
                            void *workspace, uint64_t workspace_bytes, void *stream);

/* Largest batch of gi_mlp_train_step_noalloc, and the bytes of device memory
 * its scratch takes on every GPU the library runs on (from the code object's
 * load until the process ends). */
#define GI_MLP_NOALLOC_MAX_BATCH 16384u
#define GI_MLP_NOALLOC_SCRATCH_BYTES 18355968ull

/* gi_mlp_train_step without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid allocation): the same kernels and
 * results, with the workspace in a scratch array inside the library, one
 * per GPU (its address is looked up once per device, on the first call with
 * that device current).  Allocates nothing.  n <= GI_MLP_NOALLOC_MAX_BATCH,
 * else GI_ERR_SHAPE; GI_ERR_DEVICE when the scratch cannot be located.
 * Every call on a GPU shares that GPU's scratch: calls that overlap on one
 * GPU (on different streams, or from several threads) race and must be
 * serialised by the caller.  Nothing carries over from one call to the next. */
gi_status gi_mlp_train_step_noalloc(const gi_mlp *mlp, uint32_t n, const float *pos4, const float *nrm4,
                                    const float *target4, const float *qprobe4, uint32_t t, float lr,
                                    void *stream);

/* Device workspace bytes of gi_resample_initial_mlp: 48 bytes per candidate. */
uint64_t gi_initial_mlp_workspace_bytes(uint32_t width, uint32_t height, uint32_t M);

/* gi_resample_initial with the learned cache as the target: the candidates
 * are traced (counter (pixel, frame, 0, i), as in gi_resample_initial), the
 * cache is evaluated for all of them, and the resampling uses
 * L(y) = L_e(y) + rho_y max(0, C(y, n_y)).  When the mode or the device state
 * rules the cache out, the same candidates take the probe query and the
 * result is bit-identical to gi_resample_initial.
 * Glossy scenes (GI_OPT_GLOSSY) return GI_ERR_PARAM: the cache serves Lambertian
 * scenes.  Images of more than 2^23 pixels, or W*H*M >= 2^31 candidates,
 * return GI_ERR_SHAPE. */
gi_status gi_resample_initial_mlp(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes,
                                  const gi_mlp *mlp, const gi_params *params, gi_reservoirs *out,
                                  float *resid, void *workspace, uint64_t workspace_bytes, uint64_t seed,
                                  uint32_t frame, void *stream);

/* Device workspace bytes of gi_shade_mlp: 16 bytes per pixel. */
uint64_t gi_shade_mlp_workspace_bytes(uint32_t width, uint32_t height);

/* gi_shade with the learned cache for the fresh radiance query at each
 * reservoir's sample (the cache needs no view-path bias); probe query when
 * the mode or the device state rules the cache out (then bit-identical to
 * gi_shade).
 * Glossy scenes (GI_OPT_GLOSSY) return GI_ERR_PARAM: the cache serves Lambertian
 * scenes. */
gi_status gi_shade_mlp(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes,
                       const gi_mlp *mlp, const gi_reservoirs *res, const float *resid,
                       const gi_params *params, float *out_rgba, void *workspace, uint64_t workspace_bytes,
                       void *stream);

/* Reference path tracer (converged images the estimators are compared with;
 * the paper evaluates against an unbiased path tracer, Sec. 4).  From each
 * pixel's primary vertex in gb: L = L_e(x) plus, per bounce b = 1..32, the
 * throughput times the emission hit (or the sky on a miss, which ends the
 * path); each bounce samples a cosine direction about the normal (throughput
 * *= albedo); from bounce 4 a path survives with probability P = min(1, max
 * throughput component), throughput /= P; zero albedo ends a path.  Sample
 * s, bounce b: counter (pixel, sample0 + s, 13, b).  out_rgba (float4 plane)
 * receives the mean over the spp samples (rgb, 1).  spp in 1..65536. */
gi_status gi_path_trace(const gi_scene *scene, const gi_gbuffer *gb, uint32_t spp, uint32_t sample0,
                        uint64_t seed, float *out_rgba, void *stream);

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
