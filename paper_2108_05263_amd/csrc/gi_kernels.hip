// HIP kernels and C-ABI launchers of the DDGI-resampling path (gfx950).
//
// Per-pixel kernels use 256-thread workgroups over 16x16 pixel tiles, each
// wave64 covering an 8x8 sub-tile, so SoA float4 plane accesses of a wave
// fill whole 128-byte lines and neighbouring pixels share cache lines of the
// grid, probes and reservoirs.  One kernel per C-ABI entry point; all state
// lives in caller-owned buffers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>

#include "gi.h"
#include "gi_device.hpp"
#include "gi_mlp.hpp"

using namespace gi;

namespace {

constexpr int kTile = 16;
constexpr int kBlock = 256;
constexpr uint32_t kSelBytes = 64u;   // k_initial's per-thread slot: selected candidate (3 float4), residual

// Workgroups are dealt round-robin to the chip's 8 XCDs (each with its own
// L2).  Workgroup L runs on XCD L % 8; it is given tile (L % 8) * chunk +
// L / 8 of the row-major tile order, so every XCD works through one
// contiguous band of the image and its L2 sees the scene and probes that
// band's rays reach, instead of rays from the whole frame.
#ifndef GI_XCD_BANDS
#define GI_XCD_BANDS 0
#endif
constexpr uint32_t kXcds = 8;

__device__ __forceinline__ bool tile_pixel(uint32_t W, uint32_t H, uint32_t &px, uint32_t &py)
{
    uint32_t t = threadIdx.x, w = t >> 6, l = t & 63u;
    uint32_t tx, ty;
#if GI_XCD_BANDS
    uint32_t tiles_x = (W + kTile - 1) / kTile, tiles = tiles_x * ((H + kTile - 1) / kTile);
    uint32_t chunk = (tiles + kXcds - 1) / kXcds;
    uint32_t tile = (blockIdx.x % kXcds) * chunk + blockIdx.x / kXcds;
    if (tile >= tiles) return false;
    tx = tile % tiles_x;
    ty = tile / tiles_x;
#else
    tx = blockIdx.x;
    ty = blockIdx.y;
#endif
    px = tx * kTile + (w & 1u) * 8u + (l & 7u);
    py = ty * kTile + (w >> 1) * 8u + (l >> 3);
    return px < W && py < H;
}

// Reuse passes gather from neighbours within the spatial radius: their
// workgroups are given tiles in XCD stripes, so that a pixel's neighbours
// are mostly read through one XCD's L2.  Workgroup L runs on XCD L % 8 and
// takes tile L / 8 (row-major) of stripe L % 8, a band of ceil(tx / 8) tile
// columns.
#ifndef GI_XCD_STRIPES
#define GI_XCD_STRIPES 1
#endif
__device__ __forceinline__ bool tile_pixel_striped(uint32_t W, uint32_t H, uint32_t &px, uint32_t &py)
{
#if GI_XCD_STRIPES
    const uint32_t t = threadIdx.x, w = t >> 6, l = t & 63u;
    const uint32_t tiles_x = (W + kTile - 1) / kTile;
    const uint32_t sw = (tiles_x + kXcds - 1) / kXcds;
    const uint32_t xcd = blockIdx.x % kXcds, m = blockIdx.x / kXcds;
    const uint32_t tx = xcd * sw + m % sw, ty = m / sw;
    px = tx * kTile + (w & 1u) * 8u + (l & 7u);
    py = ty * kTile + (w >> 1) * 8u + (l >> 3);
    return tx < tiles_x && px < W && py < H;
#else
    return tile_pixel(W, H, px, py);
#endif
}

dim3 tile_grid(uint32_t W, uint32_t H);

dim3 striped_grid(uint32_t W, uint32_t H)
{
#if GI_XCD_STRIPES
    const uint32_t tx = (W + kTile - 1) / kTile, ty = (H + kTile - 1) / kTile;
    const uint32_t sw = (tx + kXcds - 1) / kXcds;
    return dim3(kXcds * sw * ty);
#else
    return tile_grid(W, H);
#endif
}

dim3 tile_grid(uint32_t W, uint32_t H)
{
    uint32_t tx = (W + kTile - 1) / kTile, ty = (H + kTile - 1) / kTile;
#if GI_XCD_BANDS
    uint32_t chunk = (tx * ty + kXcds - 1) / kXcds;
    return dim3(chunk * kXcds);
#else
    return dim3(tx, ty);
#endif
}

struct GB {
    V3 pos;
    float depth;
    V3 n;
    uint32_t prim;
    V3 alb;
    float ks, rough;     // glossy layer (glossy loads only; else 0 and 1)
    V3 wo;               // unit direction toward the camera (glossy loads only)
};

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

// GLOSSY: also the glossy layer (k_s in albedo.w, roughness in emit.w) and
// the direction toward the camera position the buffer was traced from
template <bool GLOSSY = false>
__device__ __forceinline__ GB load_gb(const gi_gbuffer &g, uint32_t p)
{
    float4 a = reinterpret_cast<const float4 *>(g.pos_depth)[p];
    GB r;
    float ks = 0.0f;
    if (g.format == GI_GB_F16) {
        const half4_t b = reinterpret_cast<const half4_t *>(g.nrm_prim)[p];
        const half4_t c = reinterpret_cast<const half4_t *>(g.albedo)[p];
        const uint32_t prim16 = __builtin_bit_cast(uint16_t, b[3]);
        // a half-precision normal is renormalised: the sampling basis and the
        // cosines assume unit length
        V3 n = v3((float)b[0], (float)b[1], (float)b[2]);
        const float nn = dot(n, n);
        if (nn > 0.0f) n = frsq(nn) * n;
        r = GB{xyz(a), a.w, n, prim16 == 0xFFFFu ? GI_MISS : prim16, v3((float)c[0], (float)c[1], (float)c[2]),
               0.0f, 1.0f, v3(0.0f, 0.0f, 1.0f)};
        ks = (float)c[3];
    } else {
        float4 b = reinterpret_cast<const float4 *>(g.nrm_prim)[p];
        float4 c = reinterpret_cast<const float4 *>(g.albedo)[p];
        r = GB{xyz(a), a.w, xyz(b), __float_as_uint(b.w), xyz(c), 0.0f, 1.0f, v3(0.0f, 0.0f, 1.0f)};
        ks = c.w;
    }
    if constexpr (GLOSSY) {
        r.ks = ks;
        r.rough = reinterpret_cast<const float4 *>(g.emit)[p].w;
        V3 v = ld3(g.eye) - r.pos;
        r.wo = frsq(dot(v, v)) * v;
    }
    return r;
}

// normal + primitive and albedo (+ glossy weight k_s) records of the G-buffer's format
__device__ __forceinline__ void store_gb_na(const gi_gbuffer &g, uint32_t p, V3 n, uint32_t prim, V3 alb, float ks)
{
    if (g.format == GI_GB_F16) {
        const uint16_t prim16 = prim == GI_MISS ? (uint16_t)0xFFFFu : (uint16_t)prim;
        half4_t b = {(_Float16)n.x, (_Float16)n.y, (_Float16)n.z, __builtin_bit_cast(_Float16, prim16)};
        half4_t c = {(_Float16)alb.x, (_Float16)alb.y, (_Float16)alb.z, (_Float16)ks};
        reinterpret_cast<half4_t *>(g.nrm_prim)[p] = b;
        reinterpret_cast<half4_t *>(g.albedo)[p] = c;
        return;
    }
    reinterpret_cast<float4 *>(g.nrm_prim)[p] = make_float4(n.x, n.y, n.z, __uint_as_float(prim));
    reinterpret_cast<float4 *>(g.albedo)[p] = make_float4(alb.x, alb.y, alb.z, ks);
}

// a pixel is shaded when its surface reflects: diffuse albedo (or a glossy layer)
template <bool GLOSSY = false>
__device__ __forceinline__ bool active(const GB &g)
{
    return g.prim != GI_MISS && (!is_zero(g.alb) || (GLOSSY && g.ks > 0.0f));
}

__device__ __forceinline__ bool similar(const GB &g, const GB &q, const gi_params &pp)
{
    if (q.prim == GI_MISS) return false;
    if (dot(g.n, q.n) < pp.cos_n) return false;
    if (fabsf(g.depth - q.depth) > pp.depth_rel * g.depth) return false;
    return true;
}

// p_hat with the full BSDF of a glossy pixel: f(x, wo, wi) L min(G, G_max)
// (sky samples: f L cos)
__device__ __forceinline__ float target_glossy(const GB &g, V3 y, V3 ny, V3 L, float g_max)
{
    if (is_zero(ny)) {
        const float cx = dot(g.n, y);
        if (cx <= 0.0f) return 0.0f;
        return lum(bsdf(g.alb, g.ks, g.rough, g.n, g.wo, y) * L) * cx;
    }
    V3 v = y - g.pos;
    float d2 = dot(v, v);
    V3 w = frsq(d2) * v;
    float cx = dot(g.n, w), cy = -dot(ny, w);
    if (cx <= 0.0f || cy <= 0.0f) return 0.0f;
    return lum(bsdf(g.alb, g.ks, g.rough, g.n, g.wo, w) * L) * fminf(cx * cy * rcp(d2), g_max);
}

template <bool GLOSSY = false>
__device__ __forceinline__ float res_target(const GB &g, const Res &r, float g_max)
{
    if constexpr (GLOSSY) return target_glossy(g, r.y, r.n, r.L, g_max);
    return target(g.pos, g.n, g.alb, r.y, r.n, r.L, g_max);
}

// area density of emitter sampling at a point of primitive prim: 1/(n 4 pi r^2)
// on a listed emitter, else 0
__device__ __forceinline__ float light_pdf(const gi_scene &sc, uint32_t prim)
{
    for (uint32_t e = 0; e < sc.n_emitters; ++e)
        if (sc.emitters[e] == prim) {
            const float rad = reinterpret_cast<const float4 *>(sc.prims)[4 * prim + 1].x;
            return rcp((float)sc.n_emitters * 4.0f * kPi * rad * rad);
        }
    return 0.0f;
}

// --------------------------------------------------------------------------
// primary vertices
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_gbuffer(gi_scene sc, gi_camera cam, gi_gbuffer gb)
{
    uint32_t px, py;
    if (!tile_pixel(cam.width, cam.height, px, py)) return;
    uint32_t p = py * cam.width + px;
    float aspect = (float)cam.width / (float)cam.height;
    float sx = (2.0f * ((float)px + 0.5f) / (float)cam.width - 1.0f) * cam.tan_half_fovy * aspect;
    float sy = (1.0f - 2.0f * ((float)py + 0.5f) / (float)cam.height) * cam.tan_half_fovy;
    V3 d = ld3(cam.fwd) + sx * ld3(cam.right) + sy * ld3(cam.up);
    d = rsqrtf(dot(d, d)) * d;
    V3 o = ld3(cam.eye);
    Hit h;
    const GeoGlobal acc(sc);
    float4 *pd = reinterpret_cast<float4 *>(gb.pos_depth);
    float4 *em = reinterpret_cast<float4 *>(gb.emit);
    const V3 zero = v3(0.0f, 0.0f, 0.0f);
    if (!cast<false>(sc, acc, o, d, kInf, h)) {
        pd[p] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        store_gb_na(gb, p, zero, GI_MISS, zero, 0.0f);
        em[p] = make_float4(sc.sky[0], sc.sky[1], sc.sky[2], 1.0f);
        return;
    }
    V3 x = madd(o, h.t, d);
    V3 n = hit_normal(sc, acc, o, d, h);
    V3 alb, emit;
    float ks = 0.0f, rough = 1.0f;
    if (sc.options & GI_OPT_GLOSSY) material_g(sc, h.prim, alb, emit, ks, rough);
    else material(sc, h.prim, alb, emit);
    pd[p] = make_float4(x.x, x.y, x.z, h.t * dot(d, ld3(cam.fwd)));
    store_gb_na(gb, p, n, h.prim, alb, ks);
    em[p] = make_float4(emit.x, emit.y, emit.z, rough);
}

// --------------------------------------------------------------------------
// probe update: one workgroup per probe
// --------------------------------------------------------------------------
constexpr int kProbeBlock = 256;

// Interior texel (row-major index into the N x N interior) that padded texel
// (x, y) shows: the interior itself, or for a gutter texel the interior texel
// mirrored along the tile edge (applied first across rows, then across
// columns, which maps a corner to the diagonally opposite interior corner).
__device__ __forceinline__ int gutter_source(int x, int y, int N)
{
    int sx = x, sy = y;
    if (sy == 0 || sy == N + 1) { sx = N + 1 - sx; sy = sy == 0 ? 1 : N; }
    if (sx == 0 || sx == N + 1) { sy = N + 1 - sy; sx = sx == 0 ? 1 : N; }
    return (sy - 1) * N + (sx - 1);
}

// GLOSSY: a hit on a glossy surface adds the glossy part of L_DDGI+ toward the
// probe (Eq. 6, one lobe sample, counter (probe, frame, 15, ray))
// F16: the volume's texel format is binary16 (else FP32)
template <bool LDS, bool GLOSSY, bool F16>
__global__ void __launch_bounds__(kProbeBlock)
    k_probe_update(gi_scene sc, gi_probes in, gi_probes out, gi_probe_params pp, uint64_t seed, uint32_t frame)
{
    using Acc = typename std::conditional<LDS, GeoLds, GeoGlobal>::type;
    using F = ProbeFmt<F16>;
    if (LDS) stage_scene(sc);
    const Acc acc(sc);
    __shared__ float s_dir[GI_MAX_PROBE_RAYS][3];
    __shared__ float s_L[GI_MAX_PROBE_RAYS][3];
    __shared__ float s_d[GI_MAX_PROBE_RAYS];
    __shared__ float s_irr[8 * 8][3];
    __shared__ float s_dep[16 * 16][2];
    const uint32_t pi = blockIdx.x;
    const uint32_t ix = pi % in.dims[0], iy = (pi / in.dims[0]) % in.dims[1], iz = pi / (in.dims[0] * in.dims[1]);
    const V3 P = v3(in.lo[0] + ((float)ix + 0.5f) * in.spacing[0], in.lo[1] + ((float)iy + 0.5f) * in.spacing[1],
                    in.lo[2] + ((float)iz + 0.5f) * in.spacing[2]);
    const uint32_t R = pp.rays;
    for (uint32_t r = threadIdx.x; r < R; r += kProbeBlock) {
        uint4 rn = philox(seed, pi, frame, kPassProbe, r);
        V3 w = sphere_dir(u01(rn.x), u01(rn.y));
        Hit h;
        V3 L;
        float dist;
        if (cast<false>(sc, acc, P, w, kInf, h)) {
            V3 hp = madd(P, h.t, w);
            V3 n = hit_normal(sc, acc, P, w, h);
            V3 alb, emit;
            float ks = 0.0f, ra = 1.0f;
            if (GLOSSY) material_g(sc, h.prim, alb, emit, ks, ra);
            else material(sc, h.prim, alb, emit);
            if (pp.distance_slider > 0.0f && !is_zero(emit)) {
                // distance heuristic: emission scaled by (t / (t + s d_b))^2, d_b the
                // probe's backward mean depth clipped to its cell
                const float2 m = fetch_dep<F16>(reinterpret_cast<const char *>(in.dep) + (size_t)pi * F::kDepProbe, -w);
                float clip = kInf;
                if (w.x != 0.0f) clip = fminf(clip, 0.5f * in.spacing[0] / fabsf(w.x));
                if (w.y != 0.0f) clip = fminf(clip, 0.5f * in.spacing[1] / fabsf(w.y));
                if (w.z != 0.0f) clip = fminf(clip, 0.5f * in.spacing[2] / fabsf(w.z));
                const float db = fminf(fmaxf(m.x, 0.0f), clip);
                const float ratio = h.t / (h.t + pp.distance_slider * db);
                emit = (ratio * ratio) * emit;
            }
            L = emit;
            if (!is_zero(alb)) {
                V3 q = probe_query_fmt<1, F16>(in, view_bias(hp, P, in.bias_dist), n);
                L = v3(fmaf(alb.x, q.x, emit.x), fmaf(alb.y, q.y, emit.y), fmaf(alb.z, q.z, emit.z));
            }
            if (GLOSSY && ks > 0.0f) {
                const uint4 rg = philox(seed, pi, frame, kPassGlossyProbe, r);
                L = L + glossy_term<kTexOf<F16>>(in, view_bias(hp, P, in.bias_dist), n, -w, ks, ra, u01(rg.x), u01(rg.y));
            }
            dist = fminf(h.t, in.d_max);
        } else {
            L = ld3(sc.sky);
            dist = in.d_max;
        }
        s_dir[r][0] = w.x;
        s_dir[r][1] = w.y;
        s_dir[r][2] = w.z;
        s_L[r][0] = L.x;
        s_L[r][1] = L.y;
        s_L[r][2] = L.z;
        s_d[r] = dist;
    }
    __syncthreads();
    // old interior texel (i, j) = first texel of quad record (i+1, j+1)
    // irradiance records are quad-major: record q of probe pi is record q * nP + pi
    const size_t nP = (size_t)in.dims[0] * in.dims[1] * in.dims[2];
    const char *iold = reinterpret_cast<const char *>(in.irr) + F::kIrrRec * (size_t)pi;
    const char *dold = reinterpret_cast<const char *>(in.dep) + F::kDepProbe * (size_t)pi;
    const float hy = pp.hysteresis;
    {   // depth texel t (16x16)
        uint32_t t = threadIdx.x;
        uint32_t tx = t & 15u, ty = t >> 4;
        V3 nt = oct_decode(((float)tx + 0.5f) / 16.0f, ((float)ty + 0.5f) / 16.0f);
        float m1 = 0.0f, m2 = 0.0f, den = 0.0f;
        for (uint32_t r = 0; r < R; ++r) {
            float c = nt.x * s_dir[r][0] + nt.y * s_dir[r][1] + nt.z * s_dir[r][2];
            if (c > 0.0f) {
                float w = exp2f(pp.sharpness * __log2f(c));
                float d = s_d[r];
                m1 = fmaf(w, d, m1);
                m2 = fmaf(w, d * d, m2);
                den += w;
            }
        }
        // the stored old texel (first of quad (tx+1, ty+1)) as (mean, mean square);
        // the blend is kept as the format stores it (binary16: mean and variance)
        float2 ot[4];
        dep_texels<F16>(dold + F::kDepRec * (uint32_t)((ty + 1) * 17 + tx + 1), ot);
        const float2 old = ot[0];
        float n1 = den > 0.0f ? m1 / den : old.x;
        float n2 = den > 0.0f ? m2 / den : old.y;
        const float b1 = hy * old.x + (1.0f - hy) * n1, b2 = hy * old.y + (1.0f - hy) * n2;
        s_dep[t][0] = b1;
        s_dep[t][1] = F16 ? fmaf(-b1, b1, b2) : b2;
    }
    if (threadIdx.x < 64) {   // irradiance texel t (8x8)
        uint32_t t = threadIdx.x;
        uint32_t tx = t & 7u, ty = t >> 3;
        V3 nt = oct_decode(((float)tx + 0.5f) / 8.0f, ((float)ty + 0.5f) / 8.0f);
        V3 num = v3(0.0f, 0.0f, 0.0f);
        float den = 0.0f;
        for (uint32_t r = 0; r < R; ++r) {
            float c = nt.x * s_dir[r][0] + nt.y * s_dir[r][1] + nt.z * s_dir[r][2];
            if (c > 0.0f) {
                num = v3(fmaf(c, s_L[r][0], num.x), fmaf(c, s_L[r][1], num.y), fmaf(c, s_L[r][2], num.z));
                den += c;
            }
        }
        const char *orec = iold + F::kIrrRec * nP * (size_t)((ty + 1) * 9 + tx + 1);
        const float4 old = F16 ? half4_to_float4(*reinterpret_cast<const uint2 *>(orec))
                               : *reinterpret_cast<const float4 *>(orec);
        float id = 1.0f / den;
        V3 nv = den > 0.0f ? id * num : xyz(old);
        s_irr[t][0] = hy * old.x + (1.0f - hy) * nv.x;
        s_irr[t][1] = hy * old.y + (1.0f - hy) * nv.y;
        s_irr[t][2] = hy * old.z + (1.0f - hy) * nv.z;
    }
    __syncthreads();
    // write quad records: each corner is an interior texel or the interior
    // texel its gutter position mirrors
    char *iout = reinterpret_cast<char *>(out.irr) + F::kIrrRec * (size_t)pi;
    char *dout = reinterpret_cast<char *>(out.dep) + F::kDepProbe * (size_t)pi;
    for (uint32_t q = threadIdx.x; q < (uint32_t)kDepQuads; q += kProbeBlock) {
        int cx = (int)(q % 17u), cy = (int)(q / 17u);
        int s0 = gutter_source(cx, cy, kDepN), s1 = gutter_source(cx + 1, cy, kDepN);
        int s2 = gutter_source(cx, cy + 1, kDepN), s3 = gutter_source(cx + 1, cy + 1, kDepN);
        if constexpr (F16) {
            *reinterpret_cast<uint4 *>(dout + F::kDepRec * q) =
                make_uint4(pack_half2(s_dep[s0][0], s_dep[s0][1]), pack_half2(s_dep[s1][0], s_dep[s1][1]),
                           pack_half2(s_dep[s2][0], s_dep[s2][1]), pack_half2(s_dep[s3][0], s_dep[s3][1]));
        } else {
            float4 *rec = reinterpret_cast<float4 *>(dout + F::kDepRec * q);
            rec[0] = make_float4(s_dep[s0][0], s_dep[s0][1], s_dep[s1][0], s_dep[s1][1]);
            rec[1] = make_float4(s_dep[s2][0], s_dep[s2][1], s_dep[s3][0], s_dep[s3][1]);
        }
    }
    for (uint32_t q = threadIdx.x; q < (uint32_t)kIrrQuads; q += kProbeBlock) {
        int cx = (int)(q % 9u), cy = (int)(q / 9u);
        int s0 = gutter_source(cx, cy, kIrrN), s1 = gutter_source(cx + 1, cy, kIrrN);
        int s2 = gutter_source(cx, cy + 1, kIrrN), s3 = gutter_source(cx + 1, cy + 1, kIrrN);
        char *rb = iout + F::kIrrRec * nP * q;
        if constexpr (F16) {
            // binary16 (nearest even), in the order of the FP32 corners
            uint2 *rec = reinterpret_cast<uint2 *>(rb);
            rec[0] = make_uint2(pack_half2(s_irr[s0][0], s_irr[s0][1]), pack_half2(s_irr[s0][2], s_irr[s1][0]));
            rec[1] = make_uint2(pack_half2(s_irr[s1][1], s_irr[s1][2]), pack_half2(s_irr[s2][0], s_irr[s2][1]));
            rec[2] = make_uint2(pack_half2(s_irr[s2][2], s_irr[s3][0]), pack_half2(s_irr[s3][1], s_irr[s3][2]));
        } else {
            float4 *rec = reinterpret_cast<float4 *>(rb);
            rec[0] = make_float4(s_irr[s0][0], s_irr[s0][1], s_irr[s0][2], s_irr[s1][0]);
            rec[1] = make_float4(s_irr[s1][1], s_irr[s1][2], s_irr[s2][0], s_irr[s2][1]);
            rec[2] = make_float4(s_irr[s2][2], s_irr[s3][0], s_irr[s3][1], s_irr[s3][2]);
        }
    }
}

__global__ void k_probe_query(gi_probes pr, uint32_t n, const float *p, const float *nrm, float *out)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    V3 q = probe_query(pr, ld3(p + 3 * i), ld3(nrm + 3 * i));
    out[3 * i] = q.x;
    out[3 * i + 1] = q.y;
    out[3 * i + 2] = q.z;
}

// --------------------------------------------------------------------------
// initial resampling
// --------------------------------------------------------------------------
// Candidate planes of the learned-cache form of the initial pass: candidate
// i of pixel p at i*W*H + p; pos = (y or the miss direction, prim bits),
// nrm = (n_y, 0), q = cache value at (y, n_y).
struct CandWs {
    float4 *pos;
    float4 *nrm;
    float4 *q;
    uint32_t gate;   // kRunAlways, or run only when the cache is (kRunIfCache) / is not (kRunIfProbe) selected
};

// Gates of the learned cache's kernels in AUTO mode: the device decides per
// frame, so both forms are launched and the one not selected returns at once
// (a uniform exit before any barrier).
enum : uint32_t { kRunAlways = 0u, kRunIfCache = 1u, kRunIfProbe = 2u };

__device__ __forceinline__ bool gated_off(const CandWs &ws, const gi_mlp &mlp)
{
    return ws.gate != kRunAlways && (ws.gate == kRunIfCache) != mlp_selected(mlp);
}

// Traces the M candidates of every pixel into the candidate planes (the
// directions and hits k_initial computes itself in the probe form).
template <bool LDS>
__global__ void __launch_bounds__(kBlock)
    k_cand(gi_scene sc, gi_gbuffer gb, gi_params pp, CandWs ws, uint64_t seed, uint32_t frame, gi_mlp mlp)
{
    using Acc = typename std::conditional<LDS, GeoLds, GeoGlobal>::type;
    if (gated_off(ws, mlp)) return;
    uint32_t px, py;
    const bool inside = tile_pixel(gb.width, gb.height, px, py);
    if (LDS) stage_scene(sc);
    if (!inside) return;
    const Acc acc(sc);
    const uint32_t p = py * gb.width + px;
    const size_t npx = (size_t)gb.width * gb.height;
    const GB g = load_gb(gb, p);
    const float miss = __uint_as_float(GI_MISS);
    if (!active(g)) {
        for (uint32_t i = 0; i < pp.M; ++i) {
            ws.pos[i * npx + p] = make_float4(0.0f, 0.0f, 0.0f, miss);
            ws.nrm[i * npx + p] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        return;
    }
    const V3 o = madd(g.pos, sc.eps, g.n);
    for (uint32_t i = 0; i < pp.M; ++i) {
        uint4 rn = philox(seed, p, frame, kPassInitial, i);
        V3 w = cosine_dir(g.n, u01(rn.x), u01(rn.y));
        Hit h;
        float4 a, b = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (cast<false>(sc, acc, o, w, kInf, h)) {
            V3 y = madd(o, h.t, w), ny = hit_normal(sc, acc, o, w, h);
            a = make_float4(y.x, y.y, y.z, __uint_as_float(h.prim));
            b = make_float4(ny.x, ny.y, ny.z, 0.0f);
        } else {
            a = make_float4(w.x, w.y, w.z, miss);
        }
        ws.pos[i * npx + p] = a;
        ws.nrm[i * npx + p] = b;
    }
}

// Initial resampling.  WS = false: traces its candidates and queries the
// probes.  WS = true: takes the candidates from the planes k_cand wrote and,
// when the cache is selected, their cache values; otherwise the probe query
// of the same candidates, through the same arithmetic as WS = false.
// LIGHT: emitter candidates present (M_light > 0); without them the loop
// compiles to the plain cosine-candidate form.
// GLOSSY: the whole BSDF at x (Sec. 3.3): candidate directions from the
// mixture of the cosine and glossy lobes (lobe chosen by the candidate's
// fourth uniform), L_DDGI+ at the candidates with its glossy part (one lobe
// sample, counter (pixel, frame, 14, i)), weights p_hat over the mixture's
// density in area measure, residual f L (G - G_max) / p_A.
template <bool LDS, bool WS, bool LIGHT, bool GLOSSY, int TEX>
__global__ void __launch_bounds__(kBlock, 4)
    k_initial(gi_scene sc, gi_gbuffer gb, gi_probes pr, gi_params pp, gi_reservoirs out, float4 *resid,
              uint64_t seed, uint32_t frame, CandWs ws, gi_mlp mlp)
{
    using Acc = typename std::conditional<LDS, GeoLdsT<true>, GeoGlobal>::type;
    if (gated_off(ws, mlp)) return;
    uint32_t px, py;
    const bool inside = tile_pixel(gb.width, gb.height, px, py);
    if (LDS) stage_scene<true>(sc);
    if (!inside) return;
    const Acc acc(sc);
    const uint32_t p = py * gb.width + px;
    const GB g = load_gb<GLOSSY>(gb, p);
    if (!active<GLOSSY>(g)) {
        store_res(out, p, empty_res(0));
        resid[p] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return;
    }
    const V3 o = madd(g.pos, sc.eps, g.n);
    const V3 rho_pi = kInvPi * g.alb;
    const float pg_x = GLOSSY ? p_gloss(g.alb, g.ks) : 0.0f;
    const bool use_cache = WS && mlp_selected(mlp);
    const size_t npx = (size_t)gb.width * gb.height;
    const uint32_t Mt = LIGHT ? pp.M + pp.M_light : pp.M;
    // balance heuristic: weights divide by the mixture density (M p_A + M_light p_light) / Mt
    const float mixb = (float)pp.M / (float)Mt, mixl = (float)pp.M_light / (float)Mt;
    Res r = empty_res(Mt);
    float wsum = 0.0f, p_sel = 0.0f;
    bool have = false;
    // The selected candidate so far, (y, tag), (n_y, prim), (L, -), and
    // candidate 0's residual wait in this thread's LDS slot past the staged
    // scene: kept in registers across the probe query they would push the
    // loop's invariants into scratch.
    float4 *const sel = reinterpret_cast<float4 *>(reinterpret_cast<char *>(gi_lds) + (LDS ? lds_scene_bytes(sc) : 0u)) +
                        4u * threadIdx.x;
    sel[3] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    // subsampling: a pixel off the pattern draws no candidates, only the residual's
    const bool draws = pp.subsample <= 1u || ((uint64_t)px + py + frame) % pp.subsample == 0u;
    for (uint32_t i = 0; i < (draws ? Mt : 1u); ++i) {
        uint4 rn = philox(seed, p, frame, kPassInitial, i);
        float u2 = u01(rn.z);
        V3 w, y, ny = v3(0.0f, 0.0f, 0.0f), L = v3(0.0f, 0.0f, 0.0f);
        float phat = 0.0f, wi = 0.0f;
        uint32_t prim = GI_MISS;
        bool hit;
        if (LIGHT && i >= pp.M) {
            // emitter candidate: a point uniform in the area of a uniformly chosen emitter
            u2 = u01(rn.w);
            hit = sc.n_emitters > 0u;
            if (hit) {
                const uint32_t e = min((uint32_t)(u01(rn.x) * (float)sc.n_emitters), sc.n_emitters - 1u);
                prim = sc.emitters[e];
                const float4 c = reinterpret_cast<const float4 *>(sc.prims)[4 * prim];
                const float rad = reinterpret_cast<const float4 *>(sc.prims)[4 * prim + 1].x;
                const V3 d = sphere_dir(u01(rn.y), u01(rn.z));
                y = madd(xyz(c), rad, d);
                ny = d;
            }
        } else if constexpr (WS) {
            const float4 a = ws.pos[i * npx + p];
            w = xyz(a);
            hit = __float_as_uint(a.w) != GI_MISS;
            if (hit) {
                y = w;
                ny = xyz(ws.nrm[i * npx + p]);
                prim = __float_as_uint(a.w);
            }
        } else {
            bool dir_ok = true;
            if (GLOSSY && pg_x > 0.0f && u01(rn.w) < pg_x) dir_ok = ggx_sample(g.n, g.wo, g.rough, u01(rn.x), u01(rn.y), w);
            else w = cosine_dir(g.n, u01(rn.x), u01(rn.y));
            Hit h;
            hit = dir_ok && cast<false>(sc, acc, o, w, kInf, h);
            if (hit) {
                y = madd(o, h.t, w);
                ny = hit_normal(sc, acc, o, w, h);
                prim = h.prim;
            }
            if (GLOSSY && !dir_ok) w = v3(0.0f, 0.0f, 0.0f);   // no candidate: neither surface nor sky
        }
        if (hit) {
            V3 v = y - g.pos;
            float d2 = dot(v, v);
            V3 wv = frsq(d2) * v;
            float cx = dot(g.n, wv), cy = -dot(ny, wv);
            if (cx > 0.0f && cy > 0.0f) {
                if constexpr (GLOSSY) {
                    const uint4 rg = philox(seed, p, frame, kPassGlossyCand, i);
                    L = radiance_toward_g<TEX>(sc, pr, prim, y, ny, g.pos, u01(rg.x), u01(rg.y));
                    const V3 f = bsdf(g.alb, g.ks, g.rough, g.n, g.wo, wv) * L;
                    const float G = cx * cy * rcp(d2);
                    const float pA = mix_pdf(g.alb, g.ks, g.rough, g.n, g.wo, wv) * cy * rcp(d2);
                    phat = lum(f) * fminf(G, pp.g_max);
                    if (!LIGHT)
                        wi = pA > 0.0f ? phat * rcp(pA) : 0.0f;
                    else
                        wi = phat * rcp(mixb * pA + mixl * light_pdf(sc, prim));
                    if (i == 0 && G > pp.g_max && pA > 0.0f) { const V3 q = ((G - pp.g_max) * rcp(pA)) * f; sel[3] = make_float4(q.x, q.y, q.z, 0.0f); }
                } else {
                    // (binary16 records: the query unrolled over two corner pairs is the
                    // faster form here; FP32 records: one pair, which needs no spills)
                    L = (use_cache && i < pp.M) ? radiance_cached(sc, prim, ws.q[i * npx + p])
                                                : radiance_toward<TEX == kTexF16 ? 2 : 1, TEX>(sc, pr, prim, y, ny, g.pos);
                    float G = cx * cy * rcp(d2);
                    float fl = lum(rho_pi * L);
                    float iG = rcp(G);
                    phat = fl * fminf(G, pp.g_max);
                    if (!LIGHT)
                        wi = kPi * phat * iG;   // p_hat / p_A with p_A = G / pi
                    else
                        wi = phat * rcp(mixb * kInvPi * G + mixl * light_pdf(sc, prim));
                    if (i == 0 && G > pp.g_max) { const V3 q = (1.0f - pp.g_max * iG) * (g.alb * L); sel[3] = make_float4(q.x, q.y, q.z, 0.0f); }
                }
            }
        } else if ((!LIGHT || i < pp.M) && (!GLOSSY || !is_zero(w))) {
            y = w;
            L = ld3(sc.sky);
            float cx = dot(g.n, w);
            if (cx > 0.0f) {
                if constexpr (GLOSSY) {
                    phat = lum(bsdf(g.alb, g.ks, g.rough, g.n, g.wo, w) * L) * cx;
                    const float pd = mix_pdf(g.alb, g.ks, g.rough, g.n, g.wo, w);
                    wi = pd > 0.0f ? phat * rcp(pd) : 0.0f;
                } else {
                    phat = lum(rho_pi * L) * cx;
                    wi = kPi * phat * rcp(cx);
                }
                if (LIGHT) wi *= rcp(mixb);
            }
        }
        if (!draws) break;
        wsum += wi;
        if (u2 * wsum < wi) {
            have = true;
            p_sel = phat;
            sel[0] = make_float4(y.x, y.y, y.z, __uint_as_float(((p & 0x7FFFFFu) << 9) | ((i & 31u) << 4) | (frame & 15u)));
            sel[1] = make_float4(ny.x, ny.y, ny.z, __uint_as_float(prim));
            sel[2] = make_float4(L.x, L.y, L.z, 0.0f);
        }
    }
    if (have) {
        const float4 a = sel[0], b = sel[1], c = sel[2];
        r.y = xyz(a);
        r.tag = __float_as_uint(a.w);
        r.n = xyz(b);
        r.prim = __float_as_uint(b.w);
        r.L = xyz(c);
    }
    r.wsum = wsum;
    if (!draws) r = empty_res(0);
    r.W = (have && p_sel > 0.0f) ? wsum * rcp((float)Mt * p_sel) : 0.0f;
    store_res(out, p, r);
    resid[p] = sel[3];
}

// --------------------------------------------------------------------------
// reservoir merging (temporal and spatial reuse)
// --------------------------------------------------------------------------
struct Merge {
    float wsum;
    uint32_t Msum;
    bool have;
    Res sel;
};

template <bool GLOSSY = false>
__device__ __forceinline__ void merge_in(Merge &m, const GB &g, const Res &q, uint32_t Mq, float u, float g_max)
{
    float w = 0.0f;
    if (q.W > 0.0f && Mq > 0u) w = res_target<GLOSSY>(g, q, g_max) * q.W * (float)Mq;
    m.wsum += w;
    m.Msum += Mq;
    if (u * m.wsum < w) {
        m.have = true;
        m.sel = q;
    }
}

constexpr int kMaxDom = GI_MAX_K + 1;

// Normalise the merged reservoir.  Domain slot j holds M_j (0 = slot unused:
// a neighbour that was rejected or never drawn) and is loaded by dom(j);
// slot 0 is the pixel itself.  Slots are static so that the unrolled loop
// keeps everything in registers.
template <bool GLOSSY, int ND, class DomFn, class G>
__device__ __forceinline__ Res finish(const gi_scene &sc, const G &acc, const Merge &m, const GB &g,
                                      const uint32_t (&Mdom)[ND], DomFn dom, const gi_params &pp)
{
    if (!m.have) {
        Res e = empty_res(m.Msum);
        e.wsum = m.wsum;
        return e;
    }
    Res r = m.sel;
    float ph = res_target<GLOSSY>(g, r, pp.g_max);
    float Z;
    bool keep = true;
    if (pp.unbiased) {
        // W is zero unless x sees y and p_hat(y) > 0; the domains' rays only
        // decide Z, so they are cast only then (the result is the same)
        bool sky = is_zero(r.n);
        bool vis_x = ph > 0.0f && visible(sc, acc, g.pos, g.n, r.y, r.n, sky);
        keep = vis_x;
        uint32_t z = vis_x ? Mdom[0] : 0u;     // the target at x supports y (it was chosen)
        if (vis_x) {
#pragma unroll
            for (int j = 1; j < ND; ++j) {
                if (Mdom[j] == 0u) continue;
                GB q = dom(j);
                if (res_target<GLOSSY>(q, r, pp.g_max) <= 0.0f) continue;
                if (visible(sc, acc, q.pos, q.n, r.y, r.n, sky)) z += Mdom[j];
            }
        }
        Z = (float)z;
    } else {
        Z = (float)m.Msum;
    }
    r.wsum = m.wsum;
    r.M = m.Msum;
    r.W = (keep && Z > 0.0f && ph > 0.0f) ? m.wsum * rcp(Z * ph) : 0.0f;
    return r;
}

__device__ __forceinline__ int reproject(const gi_camera &c, V3 x)
{
    V3 v = x - ld3(c.eye);
    float z = dot(v, ld3(c.fwd));
    if (z <= 0.0f) return -1;
    float aspect = (float)c.width / (float)c.height;
    float sx = dot(v, ld3(c.right)) / (z * c.tan_half_fovy * aspect);
    float sy = dot(v, ld3(c.up)) / (z * c.tan_half_fovy);
    float fx = floorf((sx + 1.0f) * 0.5f * (float)c.width);
    float fy = floorf((1.0f - sy) * 0.5f * (float)c.height);
    if (!(fx >= 0.0f && fy >= 0.0f && fx < (float)c.width && fy < (float)c.height)) return -1;
    return (int)fy * (int)c.width + (int)fx;
}

// 8 and 5 waves per SIMD for the reuse passes (4 for the glossy spatial
// pass, whose extra state would spill more): their latency-bound gathers
// and walks gain more from occupancy than they lose to a few spilled values
template <bool LDS, bool GLOSSY>
__global__ void __launch_bounds__(kBlock, 8)
    k_temporal(gi_scene sc, gi_gbuffer gb, gi_gbuffer gbp, gi_camera cam_prev, gi_reservoirs cur,
               gi_reservoirs hist, gi_params pp, uint32_t m_hist_cap, gi_reservoirs out, uint64_t seed,
               uint32_t frame)
{
    using Acc = typename std::conditional<LDS, GeoLds, GeoGlobal>::type;
    uint32_t px, py;
    const bool inside = tile_pixel(gb.width, gb.height, px, py);
    if (LDS) stage_scene(sc);
    if (!inside) return;
    const Acc acc(sc);
    const uint32_t p = py * gb.width + px;
    const GB g = load_gb<GLOSSY>(gb, p);
    const Res rc = load_res(cur, p);
    if (!active<GLOSSY>(g)) {
        store_res(out, p, rc);
        return;
    }
    Merge m{0.0f, 0u, false, rc};
    uint32_t Mdom[2] = {rc.M, 0u};
    uint32_t qprev = 0u;
    merge_in<GLOSSY>(m, g, rc, rc.M, 0.0f, pp.g_max);
    int q = reproject(cam_prev, g.pos);
    if (q >= 0) {
        GB gq = load_gb<GLOSSY>(gbp, (uint32_t)q);
        if (similar(g, gq, pp)) {
            Res rh = load_res(hist, (uint32_t)q);
            const uint32_t Mh = min(rh.M, m_hist_cap);
            uint4 rn = philox(seed, p, frame, kPassTemporal, 0u);
            merge_in<GLOSSY>(m, g, rh, Mh, u01(rn.x), pp.g_max);
            Mdom[1] = Mh;
            qprev = (uint32_t)q;
        }
    }
    store_res(out, p, finish<GLOSSY>(sc, acc, m, g, Mdom, [&](int) { return load_gb<GLOSSY>(gbp, qprev); }, pp));
}

// Neighbour slots are static (KM of them, KM >= k): a slot that draws no
// pixel (off-screen, the pixel itself, j >= k) points at the pixel itself,
// so every neighbour load is in bounds and unconditional, and the loads of
// all slots can be in flight together instead of one neighbour after the
// other (the pass is bound by the latency of these gathers).
#ifndef GI_SPATIAL_WAVES
#define GI_SPATIAL_WAVES 5
#endif
template <bool LDS, bool GLOSSY, int KM>
__global__ void __launch_bounds__(kBlock, GLOSSY ? 4 : GI_SPATIAL_WAVES)
    k_spatial(gi_scene sc, gi_gbuffer gb, gi_reservoirs in, gi_params pp, uint32_t pass, gi_reservoirs out,
              uint64_t seed, uint32_t frame)
{
    using Acc = typename std::conditional<LDS, GeoLds, GeoGlobal>::type;
    uint32_t px, py;
    const bool inside = tile_pixel_striped(gb.width, gb.height, px, py);
    if (LDS) stage_scene(sc);
    if (!inside) return;
    const Acc acc(sc);
    const uint32_t W = gb.width, H = gb.height;
    const uint32_t p = py * W + px;
    const GB g = load_gb<GLOSSY>(gb, p);
    const Res rc = load_res(in, p);
    if (!active<GLOSSY>(g)) {
        store_res(out, p, rc);
        return;
    }
    // neighbour pixels: uniform in the disk (counter (pixel, frame, 2+pass, j))
    uint32_t qidx[KM + 1];
    bool drawn[KM];
    float uq[KM];
    qidx[0] = p;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        qidx[j + 1] = p;
        drawn[j] = false;
        uq[j] = 0.0f;
        if ((uint32_t)j >= pp.k) continue;
        const uint4 rn = philox(seed, p, frame, kPassSpatial0 + pass, (uint32_t)j);
        const float rad = pp.radius * fsqrt(u01(rn.x));
        const float s_ = sin_rev(u01(rn.y)), c_ = cos_rev(u01(rn.y));
        const int qx = (int)px + (int)floorf(rad * c_ + 0.5f);
        const int qy = (int)py + (int)floorf(rad * s_ + 0.5f);
        uq[j] = u01(rn.z);
        if (qx < 0 || qy < 0 || qx >= (int)W || qy >= (int)H) continue;
        if (qx == (int)px && qy == (int)py) continue;
        drawn[j] = true;
        qidx[j + 1] = (uint32_t)qy * W + (uint32_t)qx;
    }
    // geometric validation of every drawn neighbour (its normal and depth)
    bool use[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        const uint32_t q = qidx[j + 1];
        const float4 a = reinterpret_cast<const float4 *>(gb.pos_depth)[q];
        GB gq;
        gq.depth = a.w;
        if (gb.format == GI_GB_F16) {
            const GB full = load_gb<false>(gb, q);
            gq.n = full.n;
            gq.prim = full.prim;
        } else {
            const float4 b = reinterpret_cast<const float4 *>(gb.nrm_prim)[q];
            gq.n = xyz(b);
            gq.prim = __float_as_uint(b.w);
        }
        use[j] = drawn[j] && similar(g, gq, pp);
    }
    // merge the pixel's own reservoir, then the neighbours in order
    Merge m{0.0f, 0u, false, rc};
    uint32_t Mdom[KM + 1];
    Mdom[0] = rc.M;
    merge_in<GLOSSY>(m, g, rc, rc.M, 0.0f, pp.g_max);
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        const Res rq = load_res(in, qidx[j + 1]);
        Mdom[j + 1] = use[j] ? rq.M : 0u;
        if (use[j]) merge_in<GLOSSY>(m, g, rq, rq.M, uq[j], pp.g_max);
    }
    store_res(out, p, finish<GLOSSY>(sc, acc, m, g, Mdom, [&](int j) { return load_gb<GLOSSY>(gb, qidx[j]); }, pp));
}

// --------------------------------------------------------------------------
// shading
// --------------------------------------------------------------------------
// Specular recursion for shading (Sec. 3.3, Eq. 7-8) from the selected
// sample v (primitive prim, normal nv) toward prev: at each vertex the
// emission and the diffuse probe term rho Q(v_b, n_v), then one direction
// from the glossy lobe (counter (pixel, frame, 16, depth)) weighted
// k_s f_g cos / pdf.  While the footprint a = foot^2 stays within a_0 c and
// below the depth limit the direction is traced (the sky if it leaves) and
// the walk continues at the hit, adding sqrt(|z - v|^2 / (pdf cos_z)) to
// foot; otherwise the probes estimate the glossy integral (Q(v_b, wi)/2).
// The loop form carries the product of the weights so far (grey).
template <int TEX, class G>
__device__ V3 shade_glossy(const gi_scene &sc, const G &acc, const gi_probes &pr, const gi_params &pp, uint64_t seed,
                           uint32_t pixel, uint32_t frame, uint32_t prim, V3 v, V3 nv, V3 prev, float foot, float a0c)
{
    V3 L = v3(0.0f, 0.0f, 0.0f);
    float thr = 1.0f;
    for (uint32_t depth = 1; depth <= GI_MAX_GLOSSY_DEPTH; ++depth) {
        V3 alb, emit;
        float ks, a;
        material_g(sc, prim, alb, emit, ks, a);
        L = L + thr * emit;
        const V3 pb = view_bias(v, prev, pr.bias_dist);
        if (!is_zero(alb)) L = L + thr * (alb * probe_query<1, TEX>(pr, pb, nv));
        if (!(ks > 0.0f)) break;
        V3 wo = prev - v;
        wo = frsq(dot(wo, wo)) * wo;
        const uint4 rn = philox(seed, pixel, frame, kPassGlossyShade, depth);
        V3 wi;
        if (!ggx_sample(nv, wo, a, u01(rn.x), u01(rn.y), wi)) break;
        const float pdf = ggx_pdf(nv, wo, wi, a);
        if (!(pdf > 0.0f)) break;
        const float wgt = ks * ggx_eval(nv, wo, wi, a) * dot(nv, wi) * rcp(pdf);
        if (foot * foot > a0c || depth >= pp.glossy_depth) {
            L = L + (thr * 0.5f * wgt) * probe_query<1, TEX>(pr, pb, wi);
            break;
        }
        const V3 o = madd(v, sc.eps, nv);
        Hit h;
        if (!cast<false>(sc, acc, o, wi, kInf, h)) {
            L = L + (thr * wgt) * ld3(sc.sky);
            break;
        }
        const V3 z = madd(o, h.t, wi);
        const V3 nz = hit_normal(sc, acc, o, wi, h);
        const V3 dz = z - v;
        const float cz = -dot(nz, wi);
        foot += cz > 0.0f ? fsqrt(dot(dz, dz) * rcp(pdf * cz)) : kInf;
        thr *= wgt;
        prev = v;
        v = z;
        nv = nz;
        prim = h.prim;
    }
    return L;
}

// WS = true: the fresh query is the cache value q[p] evaluated at the
// reservoir's sample when the cache is selected (probe query otherwise).
// GLOSSY: f(x) replaces rho_x/pi and the fresh radiance follows the specular
// recursion, started with the footprint of the segment x -> y (density of
// the BSDF mixture at x) and a_0 c = c |x_0 - x|^2 / (4 pi cos) from the camera.
// The Lambertian kernel is held to 5 waves per SIMD (no spills).
template <bool LDS, bool WS, bool GLOSSY, int TEX>
__global__ void __launch_bounds__(kBlock, GLOSSY ? 1 : 5)
    k_shade(gi_scene sc, gi_gbuffer gb, gi_probes pr, gi_reservoirs res, const float4 *resid, gi_params pp,
            float4 *img, const float4 *q, gi_mlp mlp, uint64_t seed, uint32_t frame)
{
    using Acc = typename std::conditional<LDS, GeoLds, GeoGlobal>::type;
    uint32_t px, py;
    const bool inside = tile_pixel(gb.width, gb.height, px, py);
    if (LDS) stage_scene(sc);
    if (!inside) return;
    const Acc acc(sc);
    const uint32_t p = py * gb.width + px;
    const GB g = load_gb<GLOSSY>(gb, p);
    float4 e = reinterpret_cast<const float4 *>(gb.emit)[p];
    V3 o = xyz(e);
    if (g.prim != GI_MISS) {
        o = o + xyz(resid[p]);
        Res r = load_res(res, p);
        if (r.W > 0.0f) {
            V3 L, wd = r.y;
            float geo = 0.0f;
            bool ok = false;
            if (is_zero(r.n)) {
                geo = dot(g.n, r.y);
                if (geo > 0.0f && visible(sc, acc, g.pos, g.n, r.y, r.n, true)) {
                    L = ld3(sc.sky);
                    ok = true;
                }
            } else {
                V3 v = r.y - g.pos;
                float d2 = dot(v, v);
                V3 w = frsq(d2) * v;
                wd = w;
                float cx = dot(g.n, w), cy = -dot(r.n, w);
                if (cx > 0.0f && cy > 0.0f) {
                    geo = fminf(cx * cy * rcp(d2), pp.g_max);
                    if (visible(sc, acc, g.pos, g.n, r.y, r.n, false)) {
                        if constexpr (GLOSSY) {
                            const V3 vc = ld3(gb.eye) - g.pos;
                            const float c1 = dot(g.n, g.wo);
                            const float a0c = c1 > 0.0f ? pp.foot_c * dot(vc, vc) * rcp(4.0f * kPi * c1) : kInf;
                            const float p1 = mix_pdf(g.alb, g.ks, g.rough, g.n, g.wo, w);
                            const float foot = p1 > 0.0f ? fsqrt(d2 * rcp(p1 * cy)) : kInf;
                            L = shade_glossy<TEX>(sc, acc, pr, pp, seed, p, frame, r.prim, r.y, r.n, g.pos, foot, a0c);
                        } else {
                            L = (WS && mlp_selected(mlp)) ? radiance_cached(sc, r.prim, q[p])
                                                           : radiance_toward<1, TEX>(sc, pr, r.prim, r.y, r.n, g.pos);
                        }
                        ok = true;
                    }
                }
            }
            if (ok) {
                if constexpr (GLOSSY)
                    o = o + (geo * r.W) * (bsdf(g.alb, g.ks, g.rough, g.n, g.wo, wd) * L);
                else
                    o = o + (kInvPi * geo * r.W) * (g.alb * L);
            }
        }
    }
    img[p] = make_float4(o.x, o.y, o.z, 1.0f);
}

// --------------------------------------------------------------------------
// training samples of the learned cache
// --------------------------------------------------------------------------
// Sample j: pixel p = floor(u0 W H), candidate i = floor(u1 M) of the
// initial pass (its own counter), label gathered along (u2, u3) about n_y.
template <bool LDS>
__global__ void __launch_bounds__(kBlock)
    k_mlp_batch(gi_scene sc, gi_gbuffer gb, gi_probes pr, uint32_t M, uint32_t n, uint64_t seed, uint32_t frame,
                float4 *pos, float4 *nrm, float4 *tgt, float4 *qp)
{
    using Acc = typename std::conditional<LDS, GeoLds, GeoGlobal>::type;
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (LDS) stage_scene(sc);
    if (j >= n) return;
    const Acc acc(sc);
    const uint4 rn = philox(seed, j, frame, kPassTrainBatch, 0u);
    // floor(u W H) and floor(u M) exactly: u = (x >> 8) 2^-24
    const uint64_t npx = (uint64_t)gb.width * gb.height;
    const uint32_t p = (uint32_t)(((uint64_t)(rn.x >> 8) * npx) >> 24);
    const uint32_t i = (uint32_t)(((uint64_t)(rn.y >> 8) * M) >> 24);
    const float4 zero = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    pos[j] = zero;
    nrm[j] = zero;
    tgt[j] = zero;
    qp[j] = zero;
    const GB g = load_gb(gb, p);
    if (!active(g)) return;
    // the candidate, as the initial pass traces it
    const uint4 rc = philox(seed, p, frame, kPassInitial, i);
    const V3 w = cosine_dir(g.n, u01(rc.x), u01(rc.y));
    const V3 o = madd(g.pos, sc.eps, g.n);
    Hit hy;
    if (!cast<false>(sc, acc, o, w, kInf, hy)) return;
    const V3 y = madd(o, hy.t, w), ny = hit_normal(sc, acc, o, w, hy);
    V3 alb, emit;
    material(sc, hy.prim, alb, emit);
    if (is_zero(alb)) return;
    // its label
    const V3 wl = cosine_dir(ny, u01(rn.z), u01(rn.w));
    const V3 ol = madd(y, sc.eps, ny);
    Hit h;
    V3 L;
    if (cast<false>(sc, acc, ol, wl, kInf, h)) {
        const V3 z = madd(ol, h.t, wl);
        L = radiance_toward(sc, pr, h.prim, z, hit_normal(sc, acc, ol, wl, h), y);
    } else {
        L = ld3(sc.sky);
    }
    const V3 q = probe_query(pr, view_bias(y, g.pos, pr.bias_dist), ny);
    pos[j] = make_float4(y.x, y.y, y.z, 0.0f);
    nrm[j] = make_float4(ny.x, ny.y, ny.z, 0.0f);
    tgt[j] = make_float4(L.x, L.y, L.z, 1.0f);
    qp[j] = make_float4(q.x, q.y, q.z, 0.0f);
}

// --------------------------------------------------------------------------
// reference path tracer (converged images for the error statements)
// --------------------------------------------------------------------------
// GLOSSY: at every vertex the BSDF mixture of the initial pass (glossy lobe
// with probability k_s / (k_s + lum rho), chosen by u3), throughput times
// f cos / pdf, roulette after that product
template <bool LDS, bool GLOSSY>
__global__ void __launch_bounds__(kBlock)
    k_path_trace(gi_scene sc, gi_gbuffer gb, uint32_t spp, uint32_t s0, uint64_t seed, float4 *out)
{
    using Acc = typename std::conditional<LDS, GeoLds, GeoGlobal>::type;
    uint32_t px, py;
    const bool inside = tile_pixel(gb.width, gb.height, px, py);
    if (LDS) stage_scene(sc);
    if (!inside) return;
    const Acc acc(sc);
    const uint32_t p = py * gb.width + px;
    const GB g = load_gb<GLOSSY>(gb, p);
    const V3 e0 = xyz(reinterpret_cast<const float4 *>(gb.emit)[p]);
    V3 sum = v3(0.0f, 0.0f, 0.0f);
    for (uint32_t s = 0; s < spp; ++s) {
        V3 x = g.pos, n = g.n, rho = g.alb, L = e0, thr = v3(1.0f, 1.0f, 1.0f);
        if constexpr (GLOSSY) {
            if (g.prim == GI_MISS) {
                sum = sum + L;
                continue;
            }
            float ks = g.ks, ra = g.rough;
            V3 wo = g.wo;
            for (uint32_t b = 1; b <= 32; ++b) {
                if (is_zero(rho) && !(ks > 0.0f)) break;
                const uint4 rn = philox(seed, p, s0 + s, kPassReference, b);
                const float pg = p_gloss(rho, ks);
                V3 w;
                if (pg > 0.0f && u01(rn.w) < pg) {
                    if (!ggx_sample(n, wo, ra, u01(rn.x), u01(rn.y), w)) break;
                } else {
                    w = cosine_dir(n, u01(rn.x), u01(rn.y));
                }
                const float pd = mix_pdf(rho, ks, ra, n, wo, w);
                if (!(pd > 0.0f)) break;
                thr = thr * ((dot(n, w) * rcp(pd)) * bsdf(rho, ks, ra, n, wo, w));
                if (b >= 4) {
                    const float P = fminf(1.0f, fmaxf(thr.x, fmaxf(thr.y, thr.z)));
                    if (!(u01(rn.z) < P)) break;
                    thr = v3(thr.x / P, thr.y / P, thr.z / P);
                }
                const V3 o = madd(x, sc.eps, n);
                Hit h;
                if (!cast<false>(sc, acc, o, w, kInf, h)) {
                    L = L + thr * ld3(sc.sky);
                    break;
                }
                x = madd(o, h.t, w);
                n = hit_normal(sc, acc, o, w, h);
                wo = -w;
                V3 emit;
                material_g(sc, h.prim, rho, emit, ks, ra);
                L = L + thr * emit;
            }
            sum = sum + L;
            continue;
        }
        for (uint32_t b = 1; b <= 32; ++b) {
            if (is_zero(rho)) break;
            const uint4 rn = philox(seed, p, s0 + s, kPassReference, b);
            thr = thr * rho;
            if (b >= 4) {
                const float P = fminf(1.0f, fmaxf(thr.x, fmaxf(thr.y, thr.z)));
                if (!(u01(rn.z) < P)) break;
                thr = v3(thr.x / P, thr.y / P, thr.z / P);
            }
            const V3 w = cosine_dir(n, u01(rn.x), u01(rn.y));
            const V3 o = madd(x, sc.eps, n);
            Hit h;
            if (!cast<false>(sc, acc, o, w, kInf, h)) {
                L = L + thr * ld3(sc.sky);
                break;
            }
            x = madd(o, h.t, w);
            n = hit_normal(sc, acc, o, w, h);
            V3 emit;
            material(sc, h.prim, rho, emit);
            L = L + thr * emit;
        }
        sum = sum + L;
    }
    const float inv = 1.0f / (float)spp;
    out[p] = make_float4(sum.x * inv, sum.y * inv, sum.z * inv, 1.0f);
}

// --------------------------------------------------------------------------
// test hooks
// --------------------------------------------------------------------------
__global__ void k_philox(uint64_t seed, uint32_t n, const uint4 *ctr, uint4 *out)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint4 c = ctr[i];
    out[i] = philox(seed, c.x, c.y, c.z, c.w);
}

__global__ void k_trace(gi_scene sc, uint32_t n, const float *org, const float *dir, float4 *out, uint32_t *prim)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    V3 o = ld3(org + 3 * i), d = ld3(dir + 3 * i);
    Hit h;
    const GeoGlobal acc(sc);
    if (cast<false>(sc, acc, o, d, kInf, h)) {
        V3 nn = hit_normal(sc, acc, o, d, h);
        out[i] = make_float4(h.t, nn.x, nn.y, nn.z);
        prim[i] = h.prim;
    } else {
        out[i] = make_float4(kInf, 0.0f, 0.0f, 0.0f);
        prim[i] = GI_MISS;
    }
}

// --------------------------------------------------------------------------
// host-side validation
// --------------------------------------------------------------------------
gi_status launched()
{
    return hipGetLastError() == hipSuccess ? GI_OK : GI_ERR_LAUNCH;
}

gi_status check_scene(const gi_scene *sc)
{
    if (!sc) return GI_ERR_NULL;
    if (sc->n_prims > 0 && !sc->prims) return GI_ERR_NULL;
    if (sc->n_emitters > GI_MAX_EMITTERS) return GI_ERR_SHAPE;
    for (uint32_t e = 0; e < sc->n_emitters; ++e)
        if (sc->emitters[e] >= sc->n_prims) return GI_ERR_PARAM;
    if (!(sc->eps >= 0.0f)) return GI_ERR_PARAM;
    if (sc->cell_start) {
        if (!sc->cell_items && sc->n_items) return GI_ERR_NULL;
        if (sc->grid_res[0] == 0 || sc->grid_res[1] == 0 || sc->grid_res[2] == 0) return GI_ERR_SHAPE;
        if ((uint64_t)sc->grid_res[0] * sc->grid_res[1] * sc->grid_res[2] > (1u << 26)) return GI_ERR_SHAPE;
        for (int a = 0; a < 3; ++a)
            if (!(sc->grid_hi[a] > sc->grid_lo[a])) return GI_ERR_PARAM;
    }
    return GI_OK;
}

gi_status check_gb(const gi_gbuffer *g, uint32_t W, uint32_t H)
{
    if (!g || !g->pos_depth || !g->nrm_prim || !g->albedo || !g->emit) return GI_ERR_NULL;
    if (g->format > GI_GB_F16) return GI_ERR_PARAM;
    if (g->width != W || g->height != H) return GI_ERR_SHAPE;
    return GI_OK;
}

gi_status check_res(const gi_reservoirs *r, uint32_t W, uint32_t H)
{
    if (!r || !r->y_W || !r->n_wsum || !r->L_M || !r->tag_prim) return GI_ERR_NULL;
    if (r->width != W || r->height != H) return GI_ERR_SHAPE;
    return GI_OK;
}

bool res_alias(const gi_reservoirs *a, const gi_reservoirs *b)
{
    const void *pa[4] = {a->y_W, a->n_wsum, a->L_M, a->tag_prim};
    const void *pb[4] = {b->y_W, b->n_wsum, b->L_M, b->tag_prim};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            if (pa[i] == pb[j]) return true;
    return false;
}

gi_status check_probes(const gi_probes *p)
{
    if (!p || !p->irr || !p->dep) return GI_ERR_NULL;
    if (p->irr_res != 8 || p->dep_res != 16) return GI_ERR_SHAPE;
    if (p->dims[0] == 0 || p->dims[1] == 0 || p->dims[2] == 0) return GI_ERR_SHAPE;
    // the depth texture (the larger) must stay below 4 GiB: kernels use 32-bit byte offsets
    if ((uint64_t)p->dims[0] * p->dims[1] * p->dims[2] > kMaxProbes) return GI_ERR_SHAPE;
    for (int a = 0; a < 3; ++a)
        if (!(p->spacing[a] > 0.0f)) return GI_ERR_PARAM;
    if (p->texel != GI_TEXEL_F32 && p->texel != GI_TEXEL_F16) return GI_ERR_PARAM;
    return GI_OK;
}

gi_status check_params(const gi_params *pp)
{
    if (!pp) return GI_ERR_NULL;
    if (pp->M < 1 || pp->M > GI_MAX_M || pp->k > GI_MAX_K) return GI_ERR_PARAM;
    if (pp->M_light > GI_MAX_M - pp->M) return GI_ERR_PARAM;
    if (pp->subsample < 1) return GI_ERR_PARAM;
    if (!(pp->radius >= 0.0f) || !(pp->g_max > 0.0f) || !(pp->m_cap >= 0.0f) || !(pp->depth_rel >= 0.0f))
        return GI_ERR_PARAM;
    return GI_OK;
}

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Dynamic LDS a tracing kernel needs to stage the scene, or 0 to read it from
// global memory (no grid, staging switched off, or over budget: 40 KB keeps
// four 256-thread workgroups per CU; a kernel with static LDS stays within
// 64 KB in total).
constexpr uint32_t kLdsScene = 40u * 1024u;
constexpr uint32_t kLdsTotal = 64u * 1024u;
uint32_t scene_lds(const gi_scene *sc, uint32_t static_lds = 0)
{
    if (!sc->cell_start || sc->n_items == 0 || (sc->options & GI_OPT_NO_LDS)) return 0;
    uint32_t b = lds_scene_bytes(*sc);
    if (static_lds == 0) return b <= kLdsScene ? b : 0u;
    return b + static_lds <= kLdsTotal ? b : 0u;
}

#define GI_LAUNCH_LDS(kernel, grid, block, lds, stream, ...)                                   \
    do {                                                                                      \
        if (lds) kernel<true><<<(grid), (block), (lds), (stream)>>>(__VA_ARGS__);             \
        else kernel<false><<<(grid), (block), 0, (stream)>>>(__VA_ARGS__);                   \
    } while (0)
// k_initial with the scene staging (lds bytes, 0: none), emitter candidates,
// the glossy BSDF and the probes' texel format chosen at run time (the
// learned cache, WS, serves Lambertian scenes only and reads the texel format
// at run time: its probe queries are the emitter candidates' alone)
template <bool WS, bool LIGHT, int TEX, class... A>
void launch_initial_t(bool glossy, uint32_t lds, dim3 grid, hipStream_t st, A... a)
{
    // past the staged scene: every thread's selected-candidate slot
    const uint32_t extra = kBlock * kSelBytes;
    if (!WS && glossy) {
        if (lds) k_initial<true, WS, LIGHT, !WS, TEX><<<grid, kBlock, lds + extra, st>>>(a...);
        else k_initial<false, WS, LIGHT, !WS, TEX><<<grid, kBlock, extra, st>>>(a...);
    } else {
        if (lds) k_initial<true, WS, LIGHT, false, TEX><<<grid, kBlock, lds + extra, st>>>(a...);
        else k_initial<false, WS, LIGHT, false, TEX><<<grid, kBlock, extra, st>>>(a...);
    }
}
template <bool WS, bool LIGHT, class... A>
void launch_initial_l(bool glossy, bool f16, uint32_t lds, dim3 grid, hipStream_t st, A... a)
{
    if constexpr (WS) {
        launch_initial_t<WS, LIGHT, kTexAny>(glossy, lds, grid, st, a...);
    } else {
        if (f16) launch_initial_t<WS, LIGHT, kTexF16>(glossy, lds, grid, st, a...);
        else launch_initial_t<WS, LIGHT, kTexF32>(glossy, lds, grid, st, a...);
    }
}

// scene bytes to stage for k_initial: the scene and the selected-candidate
// slots together within kLdsScene, so that 4 workgroups share a CU
uint32_t initial_scene_lds(const gi_scene *sc)
{
    const uint32_t b = scene_lds(sc);
    return b && b + kBlock * kSelBytes <= kLdsScene ? b : 0u;
}

template <bool WS, class... A>
void launch_initial(bool light, bool glossy, bool f16, uint32_t lds, dim3 grid, hipStream_t st, A... a)
{
    if (light) launch_initial_l<WS, true>(glossy, f16, lds, grid, st, a...);
    else launch_initial_l<WS, false>(glossy, f16, lds, grid, st, a...);
}

bool glossy_scene(const gi_scene *sc) { return (sc->options & GI_OPT_GLOSSY) != 0u; }

#define GI_LAUNCH_LDS2(kernel, T2, grid, block, lds, stream, ...)                             \
    do {                                                                                      \
        if (lds) kernel<true, T2><<<(grid), (block), (lds), (stream)>>>(__VA_ARGS__);         \
        else kernel<false, T2><<<(grid), (block), 0, (stream)>>>(__VA_ARGS__);               \
    } while (0)

// kernel<LDS, GLOSSY> with both chosen at run time
template <int KM, class... A>
void launch_spatial(bool glossy, uint32_t lds, dim3 grid, hipStream_t st, A... a)
{
    if (glossy) {
        if (lds) k_spatial<true, true, KM><<<grid, kBlock, lds, st>>>(a...);
        else k_spatial<false, true, KM><<<grid, kBlock, 0, st>>>(a...);
    } else {
        if (lds) k_spatial<true, false, KM><<<grid, kBlock, lds, st>>>(a...);
        else k_spatial<false, false, KM><<<grid, kBlock, 0, st>>>(a...);
    }
}

#define GI_LAUNCH_LDS_G(kernel, glossy, grid, block, lds, stream, ...)                          \
    do {                                                                                      \
        if (glossy) GI_LAUNCH_LDS2(kernel, true, grid, block, lds, stream, __VA_ARGS__);       \
        else GI_LAUNCH_LDS2(kernel, false, grid, block, lds, stream, __VA_ARGS__);            \
    } while (0)

}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

const char *gi_status_string(gi_status s)
{
    switch (s) {
    case GI_OK: return "ok";
    case GI_ERR_NULL: return "null pointer";
    case GI_ERR_SHAPE: return "shape mismatch or size limit";
    case GI_ERR_PARAM: return "parameter out of range";
    case GI_ERR_ALIAS: return "output aliases an input";
    case GI_ERR_LAUNCH: return "kernel launch failed";
    case GI_ERR_DEVICE: return "no usable HIP device";
    }
    return "unknown status";
}

int gi_device(void)
{
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess) return -1;
    return d;
}

gi_status gi_trace_gbuffer(const gi_scene *scene, const gi_camera *cam, gi_gbuffer *out, void *stream)
{
    gi_status s;
    if (!cam || !out) return GI_ERR_NULL;
    if ((s = check_scene(scene)) != GI_OK) return s;
    if ((s = check_gb(out, cam->width, cam->height)) != GI_OK) return s;
    if (out->format == GI_GB_F16 && scene->n_prims + 6u >= 0xFFFFu) return GI_ERR_SHAPE;
    if (cam->width == 0 || cam->height == 0) return GI_OK;
    k_gbuffer<<<tile_grid(cam->width, cam->height), kBlock, 0, S(stream)>>>(*scene, *cam, *out);
    return launched();
}

gi_status gi_probe_update(const gi_scene *scene, const gi_probes *in, gi_probes *out, const gi_probe_params *pp,
                          uint64_t seed, uint32_t frame, void *stream)
{
    gi_status s;
    if (!pp || !out) return GI_ERR_NULL;
    if ((s = check_scene(scene)) != GI_OK) return s;
    if ((s = check_probes(in)) != GI_OK) return s;
    if ((s = check_probes(out)) != GI_OK) return s;
    for (int a = 0; a < 3; ++a)
        if (in->dims[a] != out->dims[a]) return GI_ERR_SHAPE;
    if (in->texel != out->texel) return GI_ERR_PARAM;
    const void *ii = in->irr, *id = in->dep, *oi = out->irr, *od = out->dep;
    if (ii == oi || id == od || ii == od || id == oi) return GI_ERR_ALIAS;
    if (pp->rays < 1 || pp->rays > GI_MAX_PROBE_RAYS) return GI_ERR_PARAM;
    if (!(pp->hysteresis >= 0.0f && pp->hysteresis <= 1.0f) || !(pp->sharpness > 0.0f)) return GI_ERR_PARAM;
    if (!(pp->distance_slider >= 0.0f)) return GI_ERR_PARAM;
    uint32_t P = in->dims[0] * in->dims[1] * in->dims[2];
    uint32_t lds = scene_lds(scene, (uint32_t)sizeof(float) * (7u * GI_MAX_PROBE_RAYS + 64u * 3u + 256u * 2u));
    const bool glossy = glossy_scene(scene), f16 = in->texel == GI_TEXEL_F16;
    const dim3 grid(P);
#define GI_PU(L, G, H) k_probe_update<L, G, H><<<grid, kProbeBlock, (L) ? lds : 0u, S(stream)>>>(*scene, *in, *out, *pp, seed, frame)
    if (lds) {
        if (glossy) { if (f16) GI_PU(true, true, true); else GI_PU(true, true, false); }
        else { if (f16) GI_PU(true, false, true); else GI_PU(true, false, false); }
    } else {
        if (glossy) { if (f16) GI_PU(false, true, true); else GI_PU(false, true, false); }
        else { if (f16) GI_PU(false, false, true); else GI_PU(false, false, false); }
    }
#undef GI_PU
    return launched();
}

gi_status gi_probe_query(const gi_probes *probes, uint32_t n, const float *p, const float *nrm, float *out,
                         void *stream)
{
    gi_status s;
    if ((s = check_probes(probes)) != GI_OK) return s;
    if (n == 0) return GI_OK;
    if (!p || !nrm || !out) return GI_ERR_NULL;
    k_probe_query<<<(n + 255) / 256, 256, 0, S(stream)>>>(*probes, n, p, nrm, out);
    return launched();
}

gi_status gi_resample_initial(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes,
                              const gi_params *params, gi_reservoirs *out, float *resid, uint64_t seed,
                              uint32_t frame, void *stream)
{
    gi_status s;
    if (!gb || !out || !resid) return GI_ERR_NULL;
    if ((s = check_scene(scene)) != GI_OK) return s;
    if ((s = check_gb(gb, gb->width, gb->height)) != GI_OK) return s;
    if ((s = check_probes(probes)) != GI_OK) return s;
    if ((s = check_params(params)) != GI_OK) return s;
    if ((s = check_res(out, gb->width, gb->height)) != GI_OK) return s;
    if ((uint64_t)gb->width * gb->height > (1u << 23)) return GI_ERR_SHAPE;   // 23-bit tag origin
    if (gb->width == 0 || gb->height == 0) return GI_OK;
    launch_initial<false>(params->M_light > 0, glossy_scene(scene), probes->texel == GI_TEXEL_F16, initial_scene_lds(scene),
                          tile_grid(gb->width, gb->height), S(stream),
                          *scene, *gb, *probes, *params, *out, reinterpret_cast<float4 *>(resid), seed, frame,
                          CandWs{}, gi_mlp{});
    return launched();
}

gi_status gi_resample_temporal(const gi_scene *scene, const gi_gbuffer *gb, const gi_gbuffer *gb_prev,
                               const gi_camera *prev_cam, const gi_reservoirs *cur_in,
                               const gi_reservoirs *history, const gi_params *params, gi_reservoirs *out,
                               uint64_t seed, uint32_t frame, void *stream)
{
    gi_status s;
    if (!gb || !gb_prev || !prev_cam || !cur_in || !history || !out) return GI_ERR_NULL;
    uint32_t W = gb->width, H = gb->height;
    if ((s = check_scene(scene)) != GI_OK) return s;
    if ((s = check_gb(gb, W, H)) != GI_OK) return s;
    if ((s = check_gb(gb_prev, W, H)) != GI_OK) return s;
    if (prev_cam->width != W || prev_cam->height != H) return GI_ERR_SHAPE;
    if ((s = check_params(params)) != GI_OK) return s;
    if ((s = check_res(cur_in, W, H)) != GI_OK) return s;
    if ((s = check_res(history, W, H)) != GI_OK) return s;
    if ((s = check_res(out, W, H)) != GI_OK) return s;
    if (res_alias(out, cur_in) || res_alias(out, history)) return GI_ERR_ALIAS;
    if (W == 0 || H == 0) return GI_OK;
    // the history's M is capped at a multiple of the candidates a drawing pixel
    // takes per frame, so pixels that drew none this frame (candidate
    // subsampling, Sec. 6) still take over their history
    const double capd = floor((double)params->m_cap * (double)(params->M + params->M_light));
    const uint32_t m_hist_cap = capd >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)capd;
    GI_LAUNCH_LDS_G(k_temporal, glossy_scene(scene), tile_grid(W, H), kBlock, scene_lds(scene), S(stream), *scene,
                    *gb, *gb_prev, *prev_cam, *cur_in, *history, *params, m_hist_cap, *out, seed, frame);
    return launched();
}

gi_status gi_resample_spatial(const gi_scene *scene, const gi_gbuffer *gb, const gi_reservoirs *in,
                              const gi_params *params, uint32_t pass, gi_reservoirs *out, uint64_t seed,
                              uint32_t frame, void *stream)
{
    gi_status s;
    if (!gb || !in || !out) return GI_ERR_NULL;
    uint32_t W = gb->width, H = gb->height;
    if ((s = check_scene(scene)) != GI_OK) return s;
    if ((s = check_gb(gb, W, H)) != GI_OK) return s;
    if ((s = check_params(params)) != GI_OK) return s;
    if ((s = check_res(in, W, H)) != GI_OK) return s;
    if ((s = check_res(out, W, H)) != GI_OK) return s;
    if (res_alias(out, in)) return GI_ERR_ALIAS;
    if (pass > 5) return GI_ERR_PARAM;
    if (W == 0 || H == 0) return GI_OK;
    // neighbour slots: 5 (the workloads' k) or GI_MAX_K
    if (params->k <= 5u)
        launch_spatial<5>(glossy_scene(scene), scene_lds(scene), striped_grid(W, H), S(stream), *scene, *gb, *in,
                          *params, pass, *out, seed, frame);
    else
        launch_spatial<(int)GI_MAX_K>(glossy_scene(scene), scene_lds(scene), striped_grid(W, H), S(stream), *scene,
                                      *gb, *in, *params, pass, *out, seed, frame);
    return launched();
}

gi_status gi_shade(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes, const gi_reservoirs *res,
                   const float *resid, const gi_params *params, float *out_rgba, uint64_t seed, uint32_t frame,
                   void *stream)
{
    gi_status s;
    if (!gb || !res || !resid || !out_rgba) return GI_ERR_NULL;
    uint32_t W = gb->width, H = gb->height;
    if ((s = check_scene(scene)) != GI_OK) return s;
    if ((s = check_gb(gb, W, H)) != GI_OK) return s;
    if ((s = check_probes(probes)) != GI_OK) return s;
    if ((s = check_params(params)) != GI_OK) return s;
    if ((s = check_res(res, W, H)) != GI_OK) return s;
    const bool glossy = glossy_scene(scene);
    if (glossy && (!(params->foot_c >= 0.0f) || params->glossy_depth < 1u || params->glossy_depth > GI_MAX_GLOSSY_DEPTH))
        return GI_ERR_PARAM;
    if (W == 0 || H == 0) return GI_OK;
    const uint32_t lds = scene_lds(scene);
    const dim3 grid = tile_grid(W, H);
    const float4 *rs = reinterpret_cast<const float4 *>(resid);
    float4 *img = reinterpret_cast<float4 *>(out_rgba);
    const bool f16 = probes->texel == GI_TEXEL_F16;
#define GI_SH(L, G, T)                                                                                   \
    k_shade<L, false, G, T><<<grid, kBlock, (L) ? lds : 0u, S(stream)>>>(*scene, *gb, *probes, *res, rs, *params, \
                                                                          img, nullptr, gi_mlp{}, seed, frame)
    if (glossy) {
        if (lds) { if (f16) GI_SH(true, true, kTexF16); else GI_SH(true, true, kTexF32); }
        else { if (f16) GI_SH(false, true, kTexF16); else GI_SH(false, true, kTexF32); }
    } else {
        if (lds) { if (f16) GI_SH(true, false, kTexF16); else GI_SH(true, false, kTexF32); }
        else { if (f16) GI_SH(false, false, kTexF16); else GI_SH(false, false, kTexF32); }
    }
#undef GI_SH
    return launched();
}

gi_status gi_mlp_make_batch(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes, uint32_t M,
                            uint32_t n, uint64_t seed, uint32_t frame, float *pos4, float *nrm4, float *target4,
                            float *qprobe4, void *stream)
{
    gi_status s;
    if (!gb) return GI_ERR_NULL;
    uint32_t W = gb->width, H = gb->height;
    if ((s = check_scene(scene)) != GI_OK) return s;
    if (glossy_scene(scene)) return GI_ERR_PARAM;   // the learned cache serves Lambertian scenes
    if ((s = check_gb(gb, W, H)) != GI_OK) return s;
    if ((s = check_probes(probes)) != GI_OK) return s;
    if (M < 1 || M > GI_MAX_M) return GI_ERR_PARAM;
    if (n > GI_MLP_MAX_BATCH) return GI_ERR_SHAPE;
    if (n == 0) return GI_OK;
    if (!pos4 || !nrm4 || !target4 || !qprobe4) return GI_ERR_NULL;
    if (W == 0 || H == 0) return GI_ERR_SHAPE;
    GI_LAUNCH_LDS(k_mlp_batch, (n + kBlock - 1) / kBlock, kBlock, scene_lds(scene), S(stream), *scene, *gb, *probes,
                  M, n, seed, frame, reinterpret_cast<float4 *>(pos4), reinterpret_cast<float4 *>(nrm4),
                  reinterpret_cast<float4 *>(target4), reinterpret_cast<float4 *>(qprobe4));
    return launched();
}

uint64_t gi_initial_mlp_workspace_bytes(uint32_t width, uint32_t height, uint32_t M)
{
    return 48ull * width * height * M;
}

gi_status gi_resample_initial_mlp(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes,
                                  const gi_mlp *mlp, const gi_params *params, gi_reservoirs *out, float *resid,
                                  void *workspace, uint64_t workspace_bytes, uint64_t seed, uint32_t frame,
                                  void *stream)
{
    gi_status s;
    if (!gb || !out || !resid || !workspace) return GI_ERR_NULL;
    uint32_t W = gb->width, H = gb->height;
    if ((s = check_scene(scene)) != GI_OK) return s;
    if (glossy_scene(scene)) return GI_ERR_PARAM;   // the learned cache serves Lambertian scenes
    if ((s = check_gb(gb, W, H)) != GI_OK) return s;
    if ((s = check_probes(probes)) != GI_OK) return s;
    if ((s = check_mlp(mlp)) != GI_OK) return s;
    if ((s = check_params(params)) != GI_OK) return s;
    if ((s = check_res(out, W, H)) != GI_OK) return s;
    if ((uint64_t)W * H > (1u << 23)) return GI_ERR_SHAPE;   // 23-bit tag origin
    const uint64_t ncand = (uint64_t)W * H * params->M;
    if (ncand >= (1ull << 31)) return GI_ERR_SHAPE;
    if (workspace_bytes < gi_initial_mlp_workspace_bytes(W, H, params->M)) return GI_ERR_SHAPE;
    if (W == 0 || H == 0) return GI_OK;
    float4 *base = reinterpret_cast<float4 *>(workspace);
    // NEVER: the probe form alone.  ALWAYS: the cache form (candidates traced
    // into the workspace, the cache evaluated on all of them, resampling with
    // the cached values).  AUTO: both, each gated on the device's usability
    // word, so that a frame the cache is not used in costs the probe form
    // (bit-identical to gi_resample_initial) and not the cache form's trace.
    if (mlp->mode != GI_MLP_NEVER) {
        const uint32_t gate = mlp->mode == GI_MLP_AUTO ? kRunIfCache : kRunAlways;
        CandWs ws{base, base + ncand, base + 2 * ncand, gate};
        GI_LAUNCH_LDS(k_cand, tile_grid(W, H), kBlock, scene_lds(scene), S(stream), *scene, *gb, *params, ws, seed,
                      frame, *mlp);
        if ((s = launched()) != GI_OK) return s;
        if ((s = mlp_infer_launch(*mlp, (uint32_t)ncand, ws.pos, ws.nrm, ws.q, true, S(stream))) != GI_OK) return s;
        launch_initial<true>(params->M_light > 0, false, probes->texel == GI_TEXEL_F16, 0u, tile_grid(W, H), S(stream), *scene, *gb, *probes,
                             *params, *out, reinterpret_cast<float4 *>(resid), seed, frame, ws, *mlp);
        if ((s = launched()) != GI_OK) return s;
    }
    if (mlp->mode != GI_MLP_ALWAYS) {
        const uint32_t gate = mlp->mode == GI_MLP_AUTO ? kRunIfProbe : kRunAlways;
        launch_initial<false>(params->M_light > 0, false, probes->texel == GI_TEXEL_F16, initial_scene_lds(scene), tile_grid(W, H), S(stream),
                              *scene, *gb, *probes, *params, *out, reinterpret_cast<float4 *>(resid), seed, frame,
                              CandWs{nullptr, nullptr, nullptr, gate}, *mlp);
    }
    return launched();
}

uint64_t gi_shade_mlp_workspace_bytes(uint32_t width, uint32_t height) { return 16ull * width * height; }

gi_status gi_shade_mlp(const gi_scene *scene, const gi_gbuffer *gb, const gi_probes *probes, const gi_mlp *mlp,
                       const gi_reservoirs *res, const float *resid, const gi_params *params, float *out_rgba,
                       void *workspace, uint64_t workspace_bytes, void *stream)
{
    gi_status s;
    if (!gb || !res || !resid || !out_rgba || !workspace) return GI_ERR_NULL;
    uint32_t W = gb->width, H = gb->height;
    if ((s = check_scene(scene)) != GI_OK) return s;
    if (glossy_scene(scene)) return GI_ERR_PARAM;   // the learned cache serves Lambertian scenes
    if ((s = check_gb(gb, W, H)) != GI_OK) return s;
    if ((s = check_probes(probes)) != GI_OK) return s;
    if ((s = check_mlp(mlp)) != GI_OK) return s;
    if ((s = check_params(params)) != GI_OK) return s;
    if ((s = check_res(res, W, H)) != GI_OK) return s;
    if (workspace_bytes < gi_shade_mlp_workspace_bytes(W, H)) return GI_ERR_SHAPE;
    if (W == 0 || H == 0) return GI_OK;
    float4 *q = reinterpret_cast<float4 *>(workspace);
    if ((s = mlp_infer_launch(*mlp, W * H, reinterpret_cast<const float4 *>(res->y_W),
                              reinterpret_cast<const float4 *>(res->n_wsum), q, true, S(stream))) != GI_OK)
        return s;
    {
        const uint32_t lds = scene_lds(scene);
        const float4 *rs = reinterpret_cast<const float4 *>(resid);
        float4 *img = reinterpret_cast<float4 *>(out_rgba);
        if (lds) k_shade<true, true, false, kTexAny><<<tile_grid(W, H), kBlock, lds, S(stream)>>>(*scene, *gb, *probes, *res, rs,
                                                                                      *params, img, q, *mlp, 0ull, 0u);
        else k_shade<false, true, false, kTexAny><<<tile_grid(W, H), kBlock, 0, S(stream)>>>(*scene, *gb, *probes, *res, rs,
                                                                                 *params, img, q, *mlp, 0ull, 0u);
    }
    return launched();
}

gi_status gi_path_trace(const gi_scene *scene, const gi_gbuffer *gb, uint32_t spp, uint32_t sample0, uint64_t seed,
                        float *out_rgba, void *stream)
{
    gi_status s;
    if (!gb || !out_rgba) return GI_ERR_NULL;
    uint32_t W = gb->width, H = gb->height;
    if ((s = check_scene(scene)) != GI_OK) return s;
    if ((s = check_gb(gb, W, H)) != GI_OK) return s;
    if (spp < 1 || spp > 65536) return GI_ERR_PARAM;
    if (W == 0 || H == 0) return GI_OK;
    GI_LAUNCH_LDS_G(k_path_trace, glossy_scene(scene), tile_grid(W, H), kBlock, scene_lds(scene), S(stream), *scene,
                    *gb, spp, sample0, seed,
                  reinterpret_cast<float4 *>(out_rgba));
    return launched();
}

gi_status gi_philox(uint64_t seed, uint32_t n, const uint32_t *ctr, uint32_t *out, void *stream)
{
    if (n == 0) return GI_OK;
    if (!ctr || !out) return GI_ERR_NULL;
    k_philox<<<(n + 255) / 256, 256, 0, S(stream)>>>(seed, n, reinterpret_cast<const uint4 *>(ctr),
                                                    reinterpret_cast<uint4 *>(out));
    return launched();
}

gi_status gi_trace_rays(const gi_scene *scene, uint32_t n, const float *org, const float *dir, float *out,
                        uint32_t *prim, void *stream)
{
    gi_status s;
    if ((s = check_scene(scene)) != GI_OK) return s;
    if (n == 0) return GI_OK;
    if (!org || !dir || !out || !prim) return GI_ERR_NULL;
    k_trace<<<(n + 255) / 256, 256, 0, S(stream)>>>(*scene, n, org, dir, reinterpret_cast<float4 *>(out), prim);
    return launched();
}

}  // extern "C"
