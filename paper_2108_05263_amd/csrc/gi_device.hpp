// Device-side primitives of the DDGI-resampling path for gfx950 (wave64).
//
// Everything here is FP32 and inlined into the kernels of gi_kernels.hip:
// Philox4x32-10, samplers, ray casting against the analytic scene (brute
// force or a uniform grid walked with a 3D-DDA), the octahedral probe
// fetch and the DDGI probe query, and the reservoir target function.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gi.h"

namespace gi {

constexpr float kPi = 3.14159265358979f;
constexpr float kInvPi = 0.318309886183791f;
constexpr float kInf = __builtin_huge_valf();

// Hardware reciprocal, square root and reciprocal square root (about 1 ulp);
// used instead of the IEEE-exact division/sqrt expansions, which cost ~10
// instructions each.  The path's tolerance against the FP64 oracle is far
// above these errors.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

// --------------------------------------------------------------------------
// small vector type
// --------------------------------------------------------------------------
struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator-(V3 a) { return v3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ V3 operator*(V3 a, V3 b) { return v3(a.x * b.x, a.y * b.y, a.z * b.z); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 madd(V3 o, float t, V3 d) { return v3(fmaf(t, d.x, o.x), fmaf(t, d.y, o.y), fmaf(t, d.z, o.z)); }
__device__ __forceinline__ float lum(V3 c) { return 0.2126f * c.x + 0.7152f * c.y + 0.0722f * c.z; }
__device__ __forceinline__ bool is_zero(V3 a) { return a.x == 0.0f && a.y == 0.0f && a.z == 0.0f; }
__device__ __forceinline__ V3 xyz(float4 a) { return v3(a.x, a.y, a.z); }
__device__ __forceinline__ V3 ld3(const float *a) { return v3(a[0], a[1], a[2]); }

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds; each round multiplies
// words 0 and 2 by the two round constants, crosses the high halves (xored
// with the neighbour word and the key) and the low halves; the key advances
// by the two Weyl constants between rounds.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3)
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one full 32x32->64 product per word (a single multiply instruction)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// 24-bit uniform in [0, 1): exact in FP32
__device__ __forceinline__ float u01(uint32_t v) { return (float)(v >> 8) * 5.9604644775390625e-08f; }

enum : uint32_t { kPassGlossyCand = 14, kPassGlossyProbe = 15, kPassGlossyShade = 16 };
enum : uint32_t { kPassInitial = 0, kPassTemporal = 1, kPassSpatial0 = 2, kPassProbe = 9, kPassTrainBatch = 10,
                   kPassReference = 13 };

// --------------------------------------------------------------------------
// samplers
// --------------------------------------------------------------------------
// sin(2 pi u), cos(2 pi u) for u in [0, 1): the hardware sine/cosine take
// their argument in revolutions
__device__ __forceinline__ float sin_rev(float u) { return __builtin_amdgcn_sinf(u); }
__device__ __forceinline__ float cos_rev(float u) { return __builtin_amdgcn_cosf(u); }

// cosine-weighted hemisphere about n in the branch-free basis of
// Duff et al. 2017 ("Building an Orthonormal Basis, Revisited")
__device__ __forceinline__ V3 cosine_dir(V3 n, float u0, float u1)
{
    float s_ = sin_rev(u0), c_ = cos_rev(u0);
    float r = fsqrt(u1);
    float lx = r * c_, ly = r * s_, lz = fsqrt(fmaxf(0.0f, 1.0f - u1));
    float sg = n.z >= 0.0f ? 1.0f : -1.0f;
    float a = -rcp(sg + n.z);
    float b = n.x * n.y * a;
    V3 t = v3(1.0f + sg * n.x * n.x * a, sg * b, -sg * n.x);
    V3 bt = v3(b, sg + n.y * n.y * a, -n.y);
    return v3(lx * t.x + ly * bt.x + lz * n.x, lx * t.y + ly * bt.y + lz * n.y, lx * t.z + ly * bt.z + lz * n.z);
}

__device__ __forceinline__ V3 sphere_dir(float u0, float u1)
{
    float z = 1.0f - 2.0f * u0;
    float s_ = sin_rev(u1), c_ = cos_rev(u1);
    float r = fsqrt(fmaxf(0.0f, 1.0f - z * z));
    return v3(r * c_, r * s_, z);
}

// --------------------------------------------------------------------------
// ray casting
// --------------------------------------------------------------------------
struct Hit {
    float t;
    uint32_t prim;
    int axis;        // face axis of a wall hit; a primitive's face comes from hit_normal
};

// nearest t > 0 of a sphere, in the cancellation-free form of Haines et al.
// 2019 ("Precision Improvements for Ray/Sphere Intersection")
__device__ __forceinline__ float isect_sphere(V3 o, V3 d, V3 c, float r)
{
    V3 f = o - c;
    float b = dot(f, d);
    V3 l = madd(f, -b, d);
    float disc = r * r - dot(l, l);
    if (disc < 0.0f) return kInf;
    float q = -(b + copysignf(fsqrt(disc), b));
    float cc = dot(f, f) - r * r;
    if (q == 0.0f) return kInf;
    float t0 = cc * rcp(q), t1 = q;
    float tn = fminf(t0, t1), tf = fmaxf(t0, t1);
    if (tn > 0.0f) return tn;
    if (tf > 0.0f) return tf;
    return kInf;
}

// slab test of the box [lo, hi]: nearest t > 0 on its surface, kInf if none.
// The face of the hit is not tracked here (box_axis recovers it for the one
// hit a walk keeps), so a test is two 3-way min/max and a select.
__device__ __forceinline__ float isect_box(V3 o, V3 inv, V3 lo, V3 hi)
{
    float ax = (lo.x - o.x) * inv.x, bx = (hi.x - o.x) * inv.x;
    float ay = (lo.y - o.y) * inv.y, by = (hi.y - o.y) * inv.y;
    float az = (lo.z - o.z) * inv.z, bz = (hi.z - o.z) * inv.z;
    float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fminf(az, bz));
    float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fmaxf(az, bz));
    float t = tn > 0.0f ? tn : tf;
    return (tn <= tf && t > 0.0f) ? t : kInf;
}

// face axis of a box hit returned by isect_box: the entry face (the first
// axis, in x, y, z order, whose slab entry equals the entry time), or the
// exit face when the origin lies inside the box
__device__ __forceinline__ int box_axis(V3 o, V3 inv, V3 lo, V3 hi)
{
    float ax = (lo.x - o.x) * inv.x, bx = (hi.x - o.x) * inv.x;
    float ay = (lo.y - o.y) * inv.y, by = (hi.y - o.y) * inv.y;
    float az = (lo.z - o.z) * inv.z, bz = (hi.z - o.z) * inv.z;
    float lx = fminf(ax, bx), ly = fminf(ay, by), lz = fminf(az, bz);
    float hx = fmaxf(ax, bx), hy = fmaxf(ay, by), hz = fmaxf(az, bz);
    int an = ly > lx ? 1 : 0;
    float tn = fmaxf(lx, ly);
    if (lz > tn) an = 2;
    tn = fmaxf(tn, lz);
    int af = hy < hx ? 1 : 0;
    if (hz < fminf(hx, hy)) af = 2;
    return tn > 0.0f ? an : af;
}

__device__ __forceinline__ float comp(V3 v, int a) { return a == 0 ? v.x : (a == 1 ? v.y : v.z); }

// exit of the room box from inside
__device__ __forceinline__ float isect_room(const gi_scene &sc, V3 o, V3 d, int &axis, uint32_t &wall)
{
    float best = kInf;
    int ba = -1;
    float dv[3] = {d.x, d.y, d.z}, ov[3] = {o.x, o.y, o.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (dv[a] == 0.0f) continue;
        float ta = ((dv[a] > 0.0f ? sc.room_hi[a] : sc.room_lo[a]) - ov[a]) * rcp(dv[a]);
        if (ta > 0.0f && ta < best) { best = ta; ba = a; }
    }
    if (ba < 0) return kInf;
    axis = ba;
    wall = sc.n_prims + 2u * (uint32_t)ba + (dv[ba] > 0.0f ? 1u : 0u);
    return best;
}

// Geometry as the intersection tests take it: a sphere as (centre, type)
// and (radius, -, -); a box as (lo corner, type) and (hi corner), the
// corners formed as centre -/+ half extent.
struct PrimGeo {
    V3 c;           // sphere centre, or box lo corner
    uint32_t type;
    V3 s;           // sphere radius in s.x, or box hi corner
};

__device__ __forceinline__ void geo_records(float4 a, float4 b, float4 &ga, float4 &gb)
{
    if (__float_as_uint(a.w) == 0u) {
        ga = a;
        gb = b;
    } else {
        ga = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w);
        gb = make_float4(a.x + b.x, a.y + b.y, a.z + b.z, b.w);
    }
}

__device__ __forceinline__ PrimGeo geo_of(float4 a, float4 b)
{
    return PrimGeo{v3(a.x, a.y, a.z), __float_as_uint(a.w), v3(b.x, b.y, b.z)};
}

__device__ __forceinline__ PrimGeo load_geo(const gi_prim *prims, uint32_t i)
{
    const float4 *p = reinterpret_cast<const float4 *>(prims + i);
    float4 ga, gb;
    geo_records(p[0], p[1], ga, gb);
    return geo_of(ga, gb);
}

// Scene access through the caller's device buffers.
struct GeoGlobal {
    const gi_prim *prims;
    const uint32_t *cells;
    const uint32_t *items;
    __device__ __forceinline__ explicit GeoGlobal(const gi_scene &sc)
        : prims(sc.prims), cells(sc.cell_start), items(sc.cell_items) {}
    __device__ __forceinline__ PrimGeo geo(uint32_t i) const { return load_geo(prims, i); }
    __device__ __forceinline__ uint32_t cell(uint32_t c) const { return cells[c]; }
    __device__ __forceinline__ uint32_t item(uint32_t j) const { return items[j]; }
    __device__ __forceinline__ bool has_grid() const { return cells != nullptr; }
    static constexpr bool kSplit = false;   // a cell's items in id order, types mixed
    __device__ __forceinline__ uint32_t mid(uint32_t) const { return 0u; }
};

// Scene access through a workgroup-local copy in LDS (see stage_scene):
// [2 float4 of geometry per primitive, as geo_records forms them]
// [cell_start: ncells+1][cell_mid: ncells][items]
// With kSplit, each cell's items are reordered in LDS so that its spheres
// come first: cell c lists spheres at [cell_start[c], cell_mid[c]) and boxes
// at [cell_mid[c], cell_start[c+1]), and a walk tests each run with one
// intersection routine instead of branching per item on its type.  The
// closest hit is the smallest (t, id) pair, so the order does not change it.
// The reordering costs a pass over the items per workgroup; it pays off in
// kernels that cast many rays per pixel.
extern __shared__ float4 gi_lds[];

template <bool kSplitCells>
struct GeoLdsT {
    uint32_t n_prims, n_cells;
    __device__ __forceinline__ explicit GeoLdsT(const gi_scene &sc)
        : n_prims(sc.n_prims), n_cells(sc.grid_res[0] * sc.grid_res[1] * sc.grid_res[2]) {}
    __device__ __forceinline__ PrimGeo geo(uint32_t i) const { return geo_of(gi_lds[2 * i], gi_lds[2 * i + 1]); }
    __device__ __forceinline__ uint32_t cell(uint32_t c) const
    {
        return reinterpret_cast<const uint32_t *>(gi_lds + 2 * n_prims)[c];
    }
    __device__ __forceinline__ uint32_t mid(uint32_t c) const
    {
        return reinterpret_cast<const uint32_t *>(gi_lds + 2 * n_prims)[n_cells + 1 + c];
    }
    __device__ __forceinline__ uint32_t item(uint32_t j) const
    {
        return reinterpret_cast<const uint32_t *>(gi_lds + 2 * n_prims)[2 * n_cells + 1 + j];
    }
    __device__ __forceinline__ bool has_grid() const { return true; }
    static constexpr bool kSplit = kSplitCells;
};
using GeoLds = GeoLdsT<false>;

// Bytes of LDS the staged scene needs (host and device agree on this layout).
__host__ __device__ __forceinline__ uint32_t lds_scene_bytes(const gi_scene &sc)
{
    uint32_t nc = sc.grid_res[0] * sc.grid_res[1] * sc.grid_res[2];
    uint32_t words = 2 * nc + 1 + sc.n_items;
    return 32u * sc.n_prims + ((4u * words + 15u) & ~15u);
}

// Cooperative copy of primitive geometry and the grid into LDS (with
// kSplit, then the per-cell partition of the items by type); every thread
// of the workgroup must call it (it ends with a barrier).
template <bool kSplit = false>
__device__ __forceinline__ void stage_scene(const gi_scene &sc)
{
    const float4 *src = reinterpret_cast<const float4 *>(sc.prims);
    const uint32_t n2 = 2u * sc.n_prims, bs = blockDim.x;
    for (uint32_t i = threadIdx.x; i < sc.n_prims; i += bs) geo_records(src[4u * i], src[4u * i + 1u], gi_lds[2u * i], gi_lds[2u * i + 1u]);
    uint32_t *w = reinterpret_cast<uint32_t *>(gi_lds + n2);
    const uint32_t ncell = sc.grid_res[0] * sc.grid_res[1] * sc.grid_res[2], nc = ncell + 1u;
    uint32_t *mids = w + nc, *items = w + nc + ncell;
    for (uint32_t i = threadIdx.x; i < nc; i += bs) w[i] = sc.cell_start[i];
    for (uint32_t i = threadIdx.x; i < sc.n_items; i += bs) items[i] = sc.cell_items[i];
    __syncthreads();
    if constexpr (kSplit) {
        // one thread per cell: swap boxes to the back of the cell's run
        for (uint32_t c = threadIdx.x; c < ncell; c += bs) {
            uint32_t j = w[c], k = w[c + 1u];
            while (j < k) {
                const uint32_t it = items[j];
                if (__float_as_uint(gi_lds[2u * it].w) == 0u) {
                    ++j;
                } else {
                    --k;
                    items[j] = items[k];
                    items[k] = it;
                }
            }
            mids[c] = j;
        }
        __syncthreads();
    }
}

// keep the lexicographically smallest (t, id): equal distances go to the
// lower id; a miss (t = inf) never counts, even when the running best is
// still the initial tmax = inf
__device__ __forceinline__ void take_hit(Hit &h, float t, uint32_t i)
{
    if (t < h.t || (t == h.t && t < kInf && i < h.prim)) {
        h.t = t;
        h.prim = i;
    }
}

// test one primitive of either type
template <class G>
__device__ __forceinline__ void test_prim(const G &acc, uint32_t i, V3 o, V3 d, V3 inv, Hit &h)
{
    PrimGeo g = acc.geo(i);
    float t = g.type == 0u ? isect_sphere(o, d, g.c, g.s.x) : isect_box(o, inv, g.c, g.s);
    take_hit(h, t, i);
}

// any surface crossing of a primitive in (0, tmax)?
template <class G>
__device__ __forceinline__ bool occludes_prim(const G &acc, uint32_t i, V3 o, V3 d, V3 inv, float tmax)
{
    PrimGeo g = acc.geo(i);
    float t = g.type == 0u ? isect_sphere(o, d, g.c, g.s.x) : isect_box(o, inv, g.c, g.s);
    return t < tmax;
}

// Ray cast: closest hit (ANY = false) or any hit (ANY = true) with t in (0, tmax).
// Walls are tested first; the grid (if present) is walked with a 3D-DDA and
// stops once the best hit lies before the current cell's exit.  Primitive
// boxes are padded when binned, so the grid walk returns the same hit as the
// brute-force loop.
template <bool ANY, class G>
__device__ __forceinline__ bool cast(const gi_scene &sc, const G &acc, V3 o, V3 d, float tmax, Hit &h)
{
    h.t = tmax;
    h.prim = GI_MISS;
    h.axis = -1;
    V3 inv = v3(rcp(d.x), rcp(d.y), rcp(d.z));
    if (!ANY && sc.has_room) {
        int axis;
        uint32_t wall;
        float tw = isect_room(sc, o, d, axis, wall);
        if (tw < h.t) { h.t = tw; h.prim = wall; h.axis = axis; }
    }
    if (!acc.has_grid()) {
        for (uint32_t i = 0; i < sc.n_prims; ++i) {
            if (ANY) {
                if (occludes_prim(acc, i, o, d, inv, tmax)) { h.prim = i; return true; }
            } else {
                test_prim(acc, i, o, d, inv, h);
            }
        }
        return h.prim != GI_MISS;
    }
    // clip to the grid box
    float t0 = 0.0f, t1 = h.t;
    {
        float ax = (sc.grid_lo[0] - o.x) * inv.x, bx = (sc.grid_hi[0] - o.x) * inv.x;
        float ay = (sc.grid_lo[1] - o.y) * inv.y, by = (sc.grid_hi[1] - o.y) * inv.y;
        float az = (sc.grid_lo[2] - o.z) * inv.z, bz = (sc.grid_hi[2] - o.z) * inv.z;
        t0 = fmaxf(t0, fmaxf(fminf(ax, bx), fmaxf(fminf(ay, by), fminf(az, bz))));
        t1 = fminf(t1, fminf(fmaxf(ax, bx), fminf(fmaxf(ay, by), fmaxf(az, bz))));
    }
    if (!(t0 <= t1)) return h.prim != GI_MISS;
    const int rx = (int)sc.grid_res[0], ry = (int)sc.grid_res[1], rz = (int)sc.grid_res[2];
    const float cxs = (sc.grid_hi[0] - sc.grid_lo[0]) / rx;
    const float cys = (sc.grid_hi[1] - sc.grid_lo[1]) / ry;
    const float czs = (sc.grid_hi[2] - sc.grid_lo[2]) / rz;
    V3 ps = madd(o, t0, d);
    int ix = min(max((int)floorf((ps.x - sc.grid_lo[0]) * ((float)rx / (sc.grid_hi[0] - sc.grid_lo[0]))), 0), rx - 1);
    int iy = min(max((int)floorf((ps.y - sc.grid_lo[1]) * ((float)ry / (sc.grid_hi[1] - sc.grid_lo[1]))), 0), ry - 1);
    int iz = min(max((int)floorf((ps.z - sc.grid_lo[2]) * ((float)rz / (sc.grid_hi[2] - sc.grid_lo[2]))), 0), rz - 1);
    const int sx = d.x >= 0.0f ? 1 : -1, sy = d.y >= 0.0f ? 1 : -1, sz = d.z >= 0.0f ? 1 : -1;
    // ray parameter of the next cell face crossed on each axis, advanced by
    // one cell's width per step; the accumulated rounding (a few ulps of t
    // per step) stays far below the 1e-3-cell padding of the binned boxes
    float nx = d.x == 0.0f ? kInf : (sc.grid_lo[0] + (float)(ix + (sx > 0)) * cxs - o.x) * inv.x;
    float ny = d.y == 0.0f ? kInf : (sc.grid_lo[1] + (float)(iy + (sy > 0)) * cys - o.y) * inv.y;
    float nz = d.z == 0.0f ? kInf : (sc.grid_lo[2] + (float)(iz + (sz > 0)) * czs - o.z) * inv.z;
    const float dx = d.x == 0.0f ? kInf : cxs * fabsf(inv.x);
    const float dy = d.y == 0.0f ? kInf : cys * fabsf(inv.y);
    const float dz = d.z == 0.0f ? kInf : czs * fabsf(inv.z);
    const int max_steps = rx + ry + rz + 3;
    // cell index, advanced by the step of the axis crossed
    int cell = ix + rx * (iy + ry * iz);
    const int cx = sx, cy = sy * rx, cz = sz * rx * ry;
    for (int step = 0; step < max_steps; ++step) {
        uint32_t b = acc.cell((uint32_t)cell), e = acc.cell((uint32_t)cell + 1u);
        if constexpr (G::kSplit) {
            // the cell's spheres, then its boxes (see GeoLdsT)
            const uint32_t m = acc.mid((uint32_t)cell);
            for (uint32_t j = b; j < m; ++j) {
                const uint32_t i = acc.item(j);
                const PrimGeo g = acc.geo(i);
                const float t = isect_sphere(o, d, g.c, g.s.x);
                if (ANY) {
                    if (t < tmax) { h.prim = i; return true; }
                } else {
                    take_hit(h, t, i);
                }
            }
            for (uint32_t j = m; j < e; ++j) {
                const uint32_t i = acc.item(j);
                const PrimGeo g = acc.geo(i);
                const float t = isect_box(o, inv, g.c, g.s);
                if (ANY) {
                    if (t < tmax) { h.prim = i; return true; }
                } else {
                    take_hit(h, t, i);
                }
            }
        } else {
            for (uint32_t j = b; j < e; ++j) {
                uint32_t i = acc.item(j);
                if (ANY) {
                    if (occludes_prim(acc, i, o, d, inv, tmax)) { h.prim = i; return true; }
                } else {
                    test_prim(acc, i, o, d, inv, h);
                }
            }
        }
        float texit = fminf(nx, fminf(ny, nz));
        if (texit >= fminf(t1, h.t)) break;
        // the axis whose face is crossed first (x, then y, on ties), without
        // branches: lanes stepping along different axes stay on one path
        const bool ax = nx <= ny && nx <= nz, ay = !ax && ny <= nz, az = !ax && !ay;
        ix += ax ? sx : 0;
        iy += ay ? sy : 0;
        iz += az ? sz : 0;
        nx += ax ? dx : 0.0f;
        ny += ay ? dy : 0.0f;
        nz += az ? dz : 0.0f;
        cell += ax ? cx : (ay ? cy : cz);
        if ((unsigned)ix >= (unsigned)rx || (unsigned)iy >= (unsigned)ry || (unsigned)iz >= (unsigned)rz) break;
    }
    return h.prim != GI_MISS;
}

// facing geometric normal of a closest hit
template <class G>
__device__ __forceinline__ V3 hit_normal(const gi_scene &sc, const G &acc, V3 o, V3 d, const Hit &h)
{
    V3 n;
    int axis = h.axis;
    PrimGeo g{};
    if (h.prim < sc.n_prims) {
        g = acc.geo(h.prim);
        if (g.type != 0u) axis = box_axis(o, v3(rcp(d.x), rcp(d.y), rcp(d.z)), g.c, g.s);
    }
    if (h.prim >= sc.n_prims || g.type != 0u) {
        float s = comp(d, axis) > 0.0f ? -1.0f : 1.0f;
        n = v3(axis == 0 ? s : 0.0f, axis == 1 ? s : 0.0f, axis == 2 ? s : 0.0f);
    } else {
        V3 p = madd(o, h.t, d);
        float ir = rcp(g.s.x);
        n = ir * (p - g.c);
        if (dot(n, d) > 0.0f) n = -n;
    }
    return n;
}

__device__ __forceinline__ void material(const gi_scene &sc, uint32_t prim, V3 &alb, V3 &emit)
{
    if (prim < sc.n_prims) {
        const float4 *p = reinterpret_cast<const float4 *>(sc.prims + prim);
        alb = xyz(p[2]);
        emit = xyz(p[3]);
    } else {
        alb = ld3(sc.wall_albedo);
        emit = ld3(sc.wall_emit);
    }
}

// mutual visibility of two surface points (eps-lifted), or of a point and
// the sky in direction b when b_is_dir
template <class G>
__device__ __forceinline__ bool visible(const gi_scene &sc, const G &acc, V3 a, V3 na, V3 b, V3 nb, bool b_is_dir)
{
    V3 o = madd(a, sc.eps, na);
    Hit h;
    if (b_is_dir) return !sc.has_room && !cast<true>(sc, acc, o, b, kInf, h);
    V3 e = madd(b, sc.eps, nb);
    V3 v = e - o;
    float dist = fsqrt(dot(v, v));
    V3 d = rcp(dist) * v;
    if (cast<true>(sc, acc, o, d, dist, h)) return false;
    if (sc.has_room) {
        int axis;
        uint32_t wall;
        if (isect_room(sc, o, d, axis, wall) < dist) return false;
    }
    return true;
}

// --------------------------------------------------------------------------
// octahedral tiles and the probe query
// --------------------------------------------------------------------------
__device__ __forceinline__ float sgnf(float v) { return v >= 0.0f ? 1.0f : -1.0f; }

// signed octahedral coordinates in [-1, 1]^2 of a direction of any length
__device__ __forceinline__ void oct_encode_signed(V3 v, float &px_, float &py_)
{
    float l1 = fabsf(v.x) + fabsf(v.y) + fabsf(v.z);
    float il = rcp(l1);
    float px = v.x * il, py = v.y * il;
    if (v.z < 0.0f) {
        float fx = (1.0f - fabsf(py)) * sgnf(px);
        float fy = (1.0f - fabsf(px)) * sgnf(py);
        px = fx;
        py = fy;
    }
    px_ = px;
    py_ = py;
}

__device__ __forceinline__ V3 oct_decode(float u, float w)
{
    float px = 2.0f * u - 1.0f, py = 2.0f * w - 1.0f;
    float z = 1.0f - fabsf(px) - fabsf(py);
    if (z < 0.0f) {
        float fx = (1.0f - fabsf(py)) * sgnf(px);
        float fy = (1.0f - fabsf(px)) * sgnf(py);
        px = fx;
        py = fy;
    }
    float il = frsq(px * px + py * py + z * z);
    return v3(px * il, py * il, z * il);
}

// Probe textures are stored as bilinear quads: record (cx, cy), cx, cy in
// [0, N], holds the four gutter-padded texels (cx, cy), (cx+1, cy),
// (cx, cy+1), (cx+1, cy+1) that a bilinear fetch between them needs, so one
// fetch is a single record instead of 4 scattered texel loads.  Two texel
// formats (gi_probes.texel):
//   FP32:     irradiance 12 floats (48 B: RGB of the 4 texels), depth
//             8 floats (32 B: mean and mean square of the 4 texels);
//   binary16: irradiance 12 halves (24 B), depth 8 halves (16 B: mean and
//             variance of the 4 texels; the mean square is rebuilt).
// Irradiance records are quad-major (record q of every probe, then record
// q + 1): a query reads the same record q from all 8 probes of its cell, and
// the x-neighbours' records then share cache lines.  Depth records, whose
// direction differs per probe, stay probe-major.
constexpr int kIrrN = 8, kDepN = 16;
constexpr int kIrrQuads = (kIrrN + 1) * (kIrrN + 1);      // 81 irradiance records per probe
constexpr int kDepQuads = (kDepN + 1) * (kDepN + 1);      // 289 depth records per probe

// Record sizes of a texel format (kF16: binary16, else FP32).  A volume of
// at most kMaxProbes probes keeps both textures under 4 GiB in either
// format, so kernels address them with 32-bit byte offsets.
template <bool kF16>
struct ProbeFmt {
    static constexpr uint32_t kIrrRec = kF16 ? 24u : 48u;
    static constexpr uint32_t kDepRec = kF16 ? 16u : 32u;
    static constexpr uint32_t kDepProbe = kDepQuads * kDepRec;     // 4624 or 9248
};
constexpr uint32_t kMaxProbes = 464000u;      // kMaxProbes * ProbeFmt<false>::kDepProbe < 2^32

// binary16 <-> FP32 (conversions to binary16 round to nearest even)
__device__ __forceinline__ float half_lo(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xFFFFu)); }
__device__ __forceinline__ float half_hi(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)); }
__device__ __forceinline__ float4 half4_to_float4(uint2 q)
{
    return make_float4(half_lo(q.x), half_hi(q.x), half_lo(q.y), half_hi(q.y));
}
__device__ __forceinline__ uint32_t pack_half2(float a, float b)
{
    const uint32_t lo = __builtin_bit_cast(uint16_t, (_Float16)a), hi = __builtin_bit_cast(uint16_t, (_Float16)b);
    return lo | (hi << 16);
}

// a depth texel stored as binary16 (mean, variance) -> (mean, mean square)
__device__ __forceinline__ float2 dep_texel(uint32_t w)
{
    const float mu = half_lo(w);
    return make_float2(mu, fmaf(mu, mu, half_hi(w)));
}

__device__ __forceinline__ float4 as_float4(uint4 v)
{
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
}

struct Bilin {
    int q;          // quad record index cy * (N + 1) + cx
    float ax, ay;   // fractional weights toward +x, +y
};

__device__ __forceinline__ Bilin bilin(V3 dir, int N)
{
    float u, w;
    oct_encode_signed(dir, u, w);
    // texel coordinate (u + 1)/2 * N + 1/2 of the signed octahedral coordinate u
    const float h = 0.5f * (float)N;
    float fx = fmaf(u, h, h + 0.5f), fy = fmaf(w, h, h + 0.5f);
    float x0 = floorf(fx), y0 = floorf(fy);
    Bilin b;
    // u, w lie in [0, 1] so x0, y0 lie in [0, N]; the clamp only guards
    // against a degenerate (zero or NaN) direction
    int ix = min(max((int)x0, 0), N), iy = min(max((int)y0, 0), N);
    b.q = iy * (N + 1) + ix;
    b.ax = fx - x0;
    b.ay = fy - y0;
    return b;
}

// The four (mean, mean square) texels of a depth record in memory
template <bool kF16>
__device__ __forceinline__ void dep_texels(const void *rec, float2 (&t)[4])
{
    const uint4 *r = reinterpret_cast<const uint4 *>(rec);
    if constexpr (kF16) {
        const uint4 q = r[0];
        t[0] = dep_texel(q.x); t[1] = dep_texel(q.y); t[2] = dep_texel(q.z); t[3] = dep_texel(q.w);
    } else {
        const float4 a = as_float4(r[0]), b = as_float4(r[1]);
        t[0] = make_float2(a.x, a.y); t[1] = make_float2(a.z, a.w);
        t[2] = make_float2(b.x, b.y); t[3] = make_float2(b.z, b.w);
    }
}

// bilinear (mean, mean square) of the depth records of one probe
template <bool kF16>
__device__ __forceinline__ float2 fetch_dep(const void *probe, V3 dir)
{
    Bilin b = bilin(dir, kDepN);
    float2 t[4];
    dep_texels<kF16>(reinterpret_cast<const char *>(probe) + ProbeFmt<kF16>::kDepRec * (uint32_t)b.q, t);
    float w00 = (1.0f - b.ax) * (1.0f - b.ay), w10 = b.ax * (1.0f - b.ay);
    float w01 = (1.0f - b.ax) * b.ay, w11 = b.ax * b.ay;
    return make_float2(w00 * t[0].x + w10 * t[1].x + w01 * t[2].x + w11 * t[3].x,
                       w00 * t[0].y + w10 * t[1].y + w01 * t[2].y + w11 * t[3].y);
}

__device__ __forceinline__ const float4 *at_bytes(const float *base, uint32_t off)
{
    return reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + off);
}

// Raw buffer view of a probe texture of `bytes` bytes: a load takes a 32-bit
// byte offset in a VGPR against the descriptor's base in SGPRs, so the query
// forms no 64-bit addresses; a load at or past `bytes` returns zeros.  The
// last word is the gfx9 raw-buffer format (32-bit data, no swizzle).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tex_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ uint4 tex_load16(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return make_uint4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ uint2 tex_load8(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
    return make_uint2(v[0], v[1]);
}

// The depth record at byte offset off as four (mean, mean square) texels
template <bool kF16>
__device__ __forceinline__ void dep_record(__amdgpu_buffer_rsrc_t r, uint32_t off, float2 (&t)[4])
{
    if constexpr (kF16) {
        const uint4 q = tex_load16(r, off);
        t[0] = dep_texel(q.x); t[1] = dep_texel(q.y); t[2] = dep_texel(q.z); t[3] = dep_texel(q.w);
    } else {
        const float4 a = as_float4(tex_load16(r, off)), b = as_float4(tex_load16(r, off + 16u));
        t[0] = make_float2(a.x, a.y); t[1] = make_float2(a.z, a.w);
        t[2] = make_float2(b.x, b.y); t[3] = make_float2(b.z, b.w);
    }
}

// The irradiance record at byte offset off as 12 floats (RGB of the four
// texels in order) in e0, e1, e2
template <bool kF16>
__device__ __forceinline__ void irr_record(__amdgpu_buffer_rsrc_t r, uint32_t off, float4 &e0, float4 &e1, float4 &e2)
{
    if constexpr (kF16) {
        const uint4 ia = tex_load16(r, off);
        const uint2 ib = tex_load8(r, off + 16u);
        e0 = half4_to_float4(make_uint2(ia.x, ia.y));
        e1 = half4_to_float4(make_uint2(ia.z, ia.w));
        e2 = half4_to_float4(ib);
    } else {
        e0 = as_float4(tex_load16(r, off));
        e1 = as_float4(tex_load16(r, off + 16u));
        e2 = as_float4(tex_load16(r, off + 32u));
    }
}

// Per-axis quantities of the query cell's two corner layers: offsets of the
// layers' probe coordinate from p, the trilinear fraction toward the upper
// layer, and the probe-index step between the layers (0 on a one-probe axis).
struct QueryAxis {
    float d0, d1, fr;
    uint32_t base, step;
};

__device__ __forceinline__ QueryAxis query_axis(float pv, float lo, float sp, int na, uint32_t stride)
{
    QueryAxis q;
    float g = (pv - lo) / sp - 0.5f;
    g = fminf(fmaxf(g, 0.0f), (float)(na - 1));
    const int b = min(max((int)floorf(g), 0), max(na - 2, 0));
    q.fr = na >= 2 ? g - (float)b : 0.0f;
    const int i1 = min(b + 1, na - 1);
    q.d0 = lo + ((float)b + 0.5f) * sp - pv;
    q.d1 = lo + ((float)i1 + 0.5f) * sp - pv;
    q.base = (uint32_t)b * stride;
    q.step = (uint32_t)(i1 - b) * stride;
    return q;
}

// Q(p, n) = E(p, n)/pi: blend of the 8 probes of p's cell, from textures
// of one texel format.  The per-axis terms are formed once.  The direction
// toward p is octahedral-encoded unnormalised (the encoding divides by its
// L1 norm).  Probe indices stay below 2^24, so byte offsets are 24-bit
// products.  kUnroll: how many of the four (y, z) corner pairs one loop
// iteration covers (a code-size / register trade made per kernel).
template <int kUnroll, bool kF16>
__device__ __forceinline__ V3 probe_query_fmt(const gi_probes &pr, V3 p, V3 n)
{
    using F = ProbeFmt<kF16>;
    const int nx = (int)pr.dims[0], ny = (int)pr.dims[1], nz = (int)pr.dims[2];
    const QueryAxis ax = query_axis(p.x, pr.lo[0], pr.spacing[0], nx, 1u);
    const QueryAxis ay = query_axis(p.y, pr.lo[1], pr.spacing[1], ny, (uint32_t)nx);
    const QueryAxis az = query_axis(p.z, pr.lo[2], pr.spacing[2], nz, (uint32_t)(nx * ny));
    const uint32_t base = ax.base + ay.base + az.base;
    const Bilin bn = bilin(n, kIrrN);
    const uint32_t np = (uint32_t)(nx * ny * nz);
    const uint32_t irr_q = F::kIrrRec * (uint32_t)bn.q * np;   // slice of record q
    const __amdgpu_buffer_rsrc_t dep_r = tex_rsrc(pr.dep, np * F::kDepProbe);
    const __amdgpu_buffer_rsrc_t irr_r = tex_rsrc(pr.irr, np * (uint32_t)kIrrQuads * F::kIrrRec);
    const float w00 = (1.0f - bn.ax) * (1.0f - bn.ay), w10 = bn.ax * (1.0f - bn.ay);
    const float w01 = (1.0f - bn.ax) * bn.ay, w11 = bn.ax * bn.ay;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f, wsum = 0.0f;
#pragma unroll kUnroll
    for (int c = 0; c < 4; ++c) {
        const bool oy = (c & 1) != 0, oz = (c & 2) != 0;
        const float dy = oy ? ay.d1 : ay.d0, dz = oz ? az.d1 : az.d0;
        const float ty = oy ? ay.fr : 1.0f - ay.fr, tz = oz ? az.fr : 1.0f - az.fr;
        const uint32_t pyz = base + (oy ? ay.step : 0u) + (oz ? az.step : 0u);
#pragma unroll
        for (int ox = 0; ox < 2; ++ox) {
            const V3 tp = v3(ox ? ax.d1 : ax.d0, dy, dz);
            const float tx = ox ? ax.fr : 1.0f - ax.fr;
            const uint32_t pi = pyz + (ox ? ax.step : 0u);
            const float r2 = dot(tp, tp);
            const bool at_probe = !(r2 > 0.0f);
            const float ir = frsq(r2);
            const float r = r2 * ir;
            const float hh = 0.5f * (1.0f + dot(n, tp) * ir);
            // depth moments toward p (a probe sitting exactly at p reads any texel, unused)
            const V3 dv = at_probe ? v3(0.0f, 0.0f, 1.0f) : -tp;
            const Bilin bd = bilin(dv, kDepN);
            float2 d[4];
            dep_record<kF16>(dep_r, __umul24(pi, F::kDepProbe) + F::kDepRec * (uint32_t)bd.q, d);
            float4 e0, e1, e2;
            irr_record<kF16>(irr_r, irr_q + __umul24(pi, F::kIrrRec), e0, e1, e2);
            const float v00 = (1.0f - bd.ax) * (1.0f - bd.ay), v10 = bd.ax * (1.0f - bd.ay);
            const float v01 = (1.0f - bd.ax) * bd.ay, v11 = bd.ax * bd.ay;
            const float mu = v00 * d[0].x + v10 * d[1].x + v01 * d[2].x + v11 * d[3].x;
            const float mu2 = v00 * d[0].y + v10 * d[1].y + v01 * d[2].y + v11 * d[3].y;
            const float var = fmaxf(fmaf(-mu, mu, mu2), pr.var_floor);
            const float dd = r - mu;
            const float cheb = var * rcp(fmaf(dd, dd, var));
            const float vis = (!at_probe && r > mu) ? cheb * cheb * cheb : 1.0f;
            const float back = at_probe ? 0.45f : hh * hh + 0.2f;
            const float wgt = tx * ty * tz * fmaxf(back * vis, 1e-6f);
            sx = fmaf(wgt, w00 * e0.x + w10 * e0.w + w01 * e1.z + w11 * e2.y, sx);
            sy = fmaf(wgt, w00 * e0.y + w10 * e1.x + w01 * e1.w + w11 * e2.z, sy);
            sz = fmaf(wgt, w00 * e0.z + w10 * e1.y + w01 * e2.x + w11 * e2.w, sz);
            wsum += wgt;
        }
    }
    const float iw = rcp(wsum);
    return v3(iw * sx, iw * sy, iw * sz);
}

// Texel format a kernel is compiled for: one of the two, or either (read
// from the volume at run time: a uniform branch, both forms in the code).
// The hot kernels take it as a template argument, so that only one form
// competes for their registers.
enum : int { kTexF32 = 0, kTexF16 = 1, kTexAny = 2 };
template <bool kF16>
constexpr int kTexOf = kF16 ? kTexF16 : kTexF32;

// Q(p, n) from the volume's textures
template <int kUnroll = 1, int kTex = kTexAny>
__device__ __forceinline__ V3 probe_query(const gi_probes &pr, V3 p, V3 n)
{
    if constexpr (kTex == kTexAny)
        return pr.texel == GI_TEXEL_F16 ? probe_query_fmt<kUnroll, true>(pr, p, n)
                                        : probe_query_fmt<kUnroll, false>(pr, p, n);
    else
        return probe_query_fmt<kUnroll, kTex == kTexF16>(pr, p, n);
}

// view-path bias: move y toward x by min(d, |x - y|/2)
__device__ __forceinline__ V3 view_bias(V3 y, V3 x, float d)
{
    V3 v = x - y;
    float d2 = dot(v, v);
    float id = frsq(d2);
    float s = fminf(d, 0.5f * d2 * id);
    return madd(y, s * id, v);
}

// L_e(y) + rho_y Q(y_b, n_y), y_b biased toward x
template <int kUnroll = 1, int kTex = kTexAny>
__device__ __forceinline__ V3 radiance_toward(const gi_scene &sc, const gi_probes &pr, uint32_t prim, V3 y, V3 ny, V3 x)
{
    V3 alb, emit;
    material(sc, prim, alb, emit);
    if (is_zero(alb)) return emit;
    V3 q = probe_query<kUnroll, kTex>(pr, view_bias(y, x, pr.bias_dist), ny);
    return v3(fmaf(alb.x, q.x, emit.x), fmaf(alb.y, q.y, emit.y), fmaf(alb.z, q.z, emit.z));
}

// L_e(y) + rho_y max(0, C) with a cache value C already evaluated at y (the
// learned cache needs no view-path bias); a non-finite C counts as 0
__device__ __forceinline__ V3 radiance_cached(const gi_scene &sc, uint32_t prim, float4 c)
{
    V3 alb, emit;
    material(sc, prim, alb, emit);
    if (is_zero(alb)) return emit;
    return v3(fmaf(alb.x, fmaxf(c.x, 0.0f), emit.x), fmaf(alb.y, fmaxf(c.y, 0.0f), emit.y),
              fmaf(alb.z, fmaxf(c.z, 0.0f), emit.z));
}

// --------------------------------------------------------------------------
// reservoirs
// --------------------------------------------------------------------------
struct Res {
    V3 y;
    float W;
    V3 n;
    float wsum;
    V3 L;
    uint32_t M;
    uint32_t tag, prim;
};

__device__ __forceinline__ Res load_res(const gi_reservoirs &r, uint32_t p)
{
    float4 a = reinterpret_cast<const float4 *>(r.y_W)[p];
    float4 b = reinterpret_cast<const float4 *>(r.n_wsum)[p];
    float4 c = reinterpret_cast<const float4 *>(r.L_M)[p];
    uint2 d = reinterpret_cast<const uint2 *>(r.tag_prim)[p];
    return Res{xyz(a), a.w, xyz(b), b.w, xyz(c), __float_as_uint(c.w), d.x, d.y};
}

__device__ __forceinline__ void store_res(const gi_reservoirs &r, uint32_t p, const Res &s)
{
    reinterpret_cast<float4 *>(r.y_W)[p] = make_float4(s.y.x, s.y.y, s.y.z, s.W);
    reinterpret_cast<float4 *>(r.n_wsum)[p] = make_float4(s.n.x, s.n.y, s.n.z, s.wsum);
    reinterpret_cast<float4 *>(r.L_M)[p] = make_float4(s.L.x, s.L.y, s.L.z, __uint_as_float(s.M));
    reinterpret_cast<uint2 *>(r.tag_prim)[p] = make_uint2(s.tag, s.prim);
}

__device__ __forceinline__ Res empty_res(uint32_t M)
{
    Res r;
    r.y = r.n = r.L = v3(0.0f, 0.0f, 0.0f);
    r.W = r.wsum = 0.0f;
    r.M = M;
    r.tag = GI_EMPTY_TAG;
    r.prim = GI_MISS;
    return r;
}

// target p_hat at (x, n_x, rho_x) for a sample with cached radiance L
// --------------------------------------------------------------------------
// glossy layer (Sec. 3.3, "microfacet models"): an isotropic GGX lobe with
// separable Smith masking and a grey weight k_s, no Fresnel term:
//   f = rho/pi + k_s D(h) G1(wo) G1(wi) / (4 (n.wo)(n.wi)),
//   D(h) = a^2 / (pi t^2),  t = (n.h)^2 (a^2 - 1) + 1 = a^2 + (1 - a^2) |n x h|^2,
//   G1(v) = 2 (n.v) / ((n.v) + sqrt(a^2 + (1 - a^2)(n.v)^2)).
// t is formed from |n x h|^2, which keeps its precision near the lobe's peak
// where (n.h)^2 is within rounding of 1.  The lobe is sampled by half vector
// with density D(h)(n.h) (Walter et al. 2007) and wi reflected about h; the
// density of wi is D(h)(n.h) / (4 |wo.h|).
// --------------------------------------------------------------------------
__device__ __forceinline__ V3 cross(V3 a, V3 b)
{
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ float ggx_D(V3 n, V3 h, float a)
{
    const V3 c = cross(n, h);
    const float a2 = a * a, t = fmaf(1.0f - a2, dot(c, c), a2);
    return a2 * rcp(kPi * t * t);
}

__device__ __forceinline__ float smith_G1(float nv, float a)
{
    const float a2 = a * a;
    return 2.0f * nv * rcp(nv + fsqrt(fmaf(1.0f - a2, nv * nv, a2)));
}

// f_g / k_s; 0 unless both directions lie above the surface
__device__ __forceinline__ float ggx_eval(V3 n, V3 wo, V3 wi, float a)
{
    const float no = dot(n, wo), ni = dot(n, wi);
    if (no <= 0.0f || ni <= 0.0f) return 0.0f;
    V3 h = wo + wi;
    h = frsq(dot(h, h)) * h;
    return ggx_D(n, h, a) * smith_G1(no, a) * smith_G1(ni, a) * rcp(4.0f * no * ni);
}

__device__ __forceinline__ float ggx_pdf(V3 n, V3 wo, V3 wi, float a)
{
    if (dot(n, wi) <= 0.0f || dot(n, wo) <= 0.0f) return 0.0f;
    V3 h = wo + wi;
    h = frsq(dot(h, h)) * h;
    const float oh = fabsf(dot(wo, h));
    return oh > 0.0f ? ggx_D(n, h, a) * dot(n, h) * rcp(4.0f * oh) : 0.0f;
}

// a direction from the lobe about wo; false (no sample) below the surface
__device__ __forceinline__ bool ggx_sample(V3 n, V3 wo, float a, float u0, float u1, V3 &wi)
{
    // cos^2 and sin^2 of theta_h: (1 - u0) / d and a^2 u0 / d, d = 1 - u0 + a^2 u0
    const float a2 = a * a, om = 1.0f - u0, d = rcp(fmaf(a2, u0, om));
    const float ct = fsqrt(om * d), st = fsqrt(a2 * u0 * d);
    const float sp = sin_rev(u1), cp = cos_rev(u1);
    const float sg = n.z >= 0.0f ? 1.0f : -1.0f;
    const float aa = -rcp(sg + n.z);
    const float b = n.x * n.y * aa;
    const V3 t = v3(1.0f + sg * n.x * n.x * aa, sg * b, -sg * n.x);
    const V3 bt = v3(b, sg + n.y * n.y * aa, -n.y);
    const V3 h = v3(st * cp * t.x + st * sp * bt.x + ct * n.x, st * cp * t.y + st * sp * bt.y + ct * n.y,
                    st * cp * t.z + st * sp * bt.z + ct * n.z);
    const float oh = dot(wo, h);
    wi = v3(2.0f * oh * h.x - wo.x, 2.0f * oh * h.y - wo.y, 2.0f * oh * h.z - wo.z);
    return dot(n, wi) > 0.0f && dot(n, wo) > 0.0f;
}

// primary-vertex lobe choice: the glossy lobe with probability k_s / (k_s + lum(rho))
__device__ __forceinline__ float p_gloss(V3 rho, float ks) { return ks > 0.0f ? ks * rcp(ks + lum(rho)) : 0.0f; }

// solid-angle density of the BSDF mixture
__device__ __forceinline__ float mix_pdf(V3 rho, float ks, float a, V3 n, V3 wo, V3 wi)
{
    const float pg = p_gloss(rho, ks), c = dot(n, wi);
    const float pd = c > 0.0f ? c * kInvPi : 0.0f;
    return (1.0f - pg) * pd + (pg > 0.0f ? pg * ggx_pdf(n, wo, wi, a) : 0.0f);
}

// f = rho/pi + k_s f_g(wo, wi)
__device__ __forceinline__ V3 bsdf(V3 rho, float ks, float a, V3 n, V3 wo, V3 wi)
{
    const float g = ks > 0.0f ? ks * ggx_eval(n, wo, wi, a) : 0.0f;
    return v3(fmaf(kInvPi, rho.x, g), fmaf(kInvPi, rho.y, g), fmaf(kInvPi, rho.z, g));
}

// material with the glossy layer (record slots albedo.w = k_s, emit.w = roughness)
__device__ __forceinline__ void material_g(const gi_scene &sc, uint32_t prim, V3 &alb, V3 &emit, float &ks, float &a)
{
    if (prim < sc.n_prims) {
        const float4 *p = reinterpret_cast<const float4 *>(sc.prims + prim);
        const float4 c = p[2], e = p[3];
        alb = xyz(c);
        emit = xyz(e);
        ks = c.w;
        a = e.w;
    } else {
        alb = ld3(sc.wall_albedo);
        emit = ld3(sc.wall_emit);
        ks = 0.0f;
        a = 1.0f;
    }
}

// glossy part of L_DDGI+ (Eq. 6): one lobe sample wi, weighted k_s f_g cos / pdf,
// times E(pb, wi)/(2 pi) = Q(pb, wi)/2 (the tiles hold E/pi; the query takes
// wi in place of the normal)
template <int kTex = kTexAny>
__device__ __forceinline__ V3 glossy_term(const gi_probes &pr, V3 pb, V3 n, V3 wo, float ks, float a, float u0, float u1)
{
    V3 wi;
    if (!ggx_sample(n, wo, a, u0, u1, wi)) return v3(0.0f, 0.0f, 0.0f);
    const float pdf = ggx_pdf(n, wo, wi, a);
    if (!(pdf > 0.0f)) return v3(0.0f, 0.0f, 0.0f);
    const float w = ks * ggx_eval(n, wo, wi, a) * dot(n, wi) * rcp(pdf);
    return (0.5f * w) * probe_query<1, kTex>(pr, pb, wi);
}

// L_DDGI+ leaving y toward x in a glossy scene: L_e + rho Q(y_b, n_y) + the
// glossy part with uniforms (u0, u1)
template <int kTex = kTexAny>
__device__ __forceinline__ V3 radiance_toward_g(const gi_scene &sc, const gi_probes &pr, uint32_t prim, V3 y, V3 ny,
                                                V3 x, float u0, float u1)
{
    V3 alb, emit;
    float ks, a;
    material_g(sc, prim, alb, emit, ks, a);
    V3 L = emit;
    const bool diff = !is_zero(alb);
    if (!diff && !(ks > 0.0f)) return L;
    const V3 pb = view_bias(y, x, pr.bias_dist);
    if (diff) {
        const V3 q = probe_query<1, kTex>(pr, pb, ny);
        L = v3(fmaf(alb.x, q.x, L.x), fmaf(alb.y, q.y, L.y), fmaf(alb.z, q.z, L.z));
    }
    if (ks > 0.0f) {
        V3 wo = x - y;
        wo = frsq(dot(wo, wo)) * wo;
        L = L + glossy_term<kTex>(pr, pb, ny, wo, ks, a, u0, u1);
    }
    return L;
}

__device__ __forceinline__ float target(V3 x, V3 nx, V3 rho, V3 y, V3 ny, V3 L, float g_max)
{
    float fl = kInvPi * lum(rho * L);
    if (is_zero(ny)) {
        float cx = dot(nx, y);
        return cx > 0.0f ? fl * cx : 0.0f;
    }
    V3 v = y - x;
    float d2 = dot(v, v);
    V3 w = frsq(d2) * v;
    float cx = dot(nx, w), cy = -dot(ny, w);
    if (cx <= 0.0f || cy <= 0.0f) return 0.0f;
    float G = cx * cy * rcp(d2);
    return fl * fminf(G, g_max);
}

}  // namespace gi
