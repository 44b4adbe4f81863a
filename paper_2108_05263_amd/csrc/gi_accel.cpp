// Host builder of the uniform-grid accelerator (see gi_accel_build_host in gi.h).
//
// Each primitive is listed in every cell its axis-aligned bounding box,
// padded by 1e-3 of a cell, overlaps.  The padding absorbs the FP32 rounding
// of the device's cell walk, so a hit point near a cell face is always found
// in the cell the walk is visiting.  Items of a cell are in increasing id
// order, which makes the build deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gi.h"

#ifndef GI_BUILD_HASH
#define GI_BUILD_HASH "unknown"
#endif

// provenance: the build script passes the hash of the sources and flags; the
// loader finds it in the file by its marker and compares it with the tree's
extern "C" __attribute__((used)) const char gi_build_id[] = "GI_BUILD_HASH=" GI_BUILD_HASH;

extern "C" const char *gi_build_hash(void) { return gi_build_id + 14; }

namespace {

void cell_range(const gi_prim &p, const float lo[3], const float cs[3], const uint32_t res[3], int c0[3], int c1[3])
{
    for (int a = 0; a < 3; ++a) {
        float half = p.type == 0u ? p.size[0] : p.size[a];
        float pad = 1e-3f * cs[a];
        float mn = p.center[a] - half - pad, mx = p.center[a] + half + pad;
        int i0 = (int)std::floor((mn - lo[a]) / cs[a]);
        int i1 = (int)std::floor((mx - lo[a]) / cs[a]);
        c0[a] = std::clamp(i0, 0, (int)res[a] - 1);
        c1[a] = std::clamp(i1, 0, (int)res[a] - 1);
        if (i1 < 0 || i0 >= (int)res[a]) c1[a] = c0[a] - 1;   // entirely outside on this axis
    }
}

}  // namespace

extern "C" gi_status gi_accel_build_host(const gi_prim *prims, uint32_t n, const float lo[3], const float hi[3],
                                         const uint32_t res[3], uint32_t *cell_start, uint32_t *items,
                                         uint32_t capacity, uint32_t *n_items)
{
    if ((n > 0 && !prims) || !lo || !hi || !res || !cell_start || !n_items) return GI_ERR_NULL;
    if (res[0] == 0 || res[1] == 0 || res[2] == 0) return GI_ERR_SHAPE;
    uint64_t ncell = (uint64_t)res[0] * res[1] * res[2];
    if (ncell > (1u << 26)) return GI_ERR_SHAPE;
    float cs[3];
    for (int a = 0; a < 3; ++a) {
        if (!(hi[a] > lo[a])) return GI_ERR_PARAM;
        cs[a] = (hi[a] - lo[a]) / (float)res[a];
    }
    std::vector<uint32_t> count(ncell + 1, 0u);
    for (uint32_t i = 0; i < n; ++i) {
        int c0[3], c1[3];
        cell_range(prims[i], lo, cs, res, c0, c1);
        for (int z = c0[2]; z <= c1[2]; ++z)
            for (int y = c0[1]; y <= c1[1]; ++y)
                for (int x = c0[0]; x <= c1[0]; ++x) ++count[(size_t)x + res[0] * ((size_t)y + res[1] * z)];
    }
    uint64_t total = 0;
    for (uint64_t c = 0; c < ncell; ++c) {
        cell_start[c] = (uint32_t)total;
        total += count[c];
    }
    cell_start[ncell] = (uint32_t)total;
    *n_items = (uint32_t)total;
    if (total > 0xFFFFFFFFull) return GI_ERR_SHAPE;
    if (total > capacity || (total > 0 && !items)) return GI_ERR_SHAPE;
    std::vector<uint32_t> fill(cell_start, cell_start + ncell);
    for (uint32_t i = 0; i < n; ++i) {
        int c0[3], c1[3];
        cell_range(prims[i], lo, cs, res, c0, c1);
        for (int z = c0[2]; z <= c1[2]; ++z)
            for (int y = c0[1]; y <= c1[1]; ++y)
                for (int x = c0[0]; x <= c1[0]; ++x) items[fill[(size_t)x + res[0] * ((size_t)y + res[1] * z)]++] = i;
    }
    return GI_OK;
}
