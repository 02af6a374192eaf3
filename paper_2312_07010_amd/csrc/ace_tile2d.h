// 2D regions for temporal blocking, shared by the blocked 2D kernels and the
// batched launch's large 2D instances: a 32 x 64 region of LDS (with a zero
// pad all around) around a (32 - 2K) x (64 - 2K) output tile, a ring of K
// nodes recomputed instead of exchanged.  Values outside the domain are
// loaded BC-mapped (clamped / zero / wrapped); for Neumann and Dirichlet an
// in-domain boundary node reads its outward neighbour from its own slot
// (mirror) or from the zero pad, since the ring slots outside the domain are
// only right at level 0.
#pragma once

#include "ace_device.h"

namespace ace {
namespace tile2d {

constexpr int BX = 64;           // region width (one wavefront)
constexpr int BH = 32;           // region height
constexpr int BLW = BX + 2;      // padded LDS row
constexpr int BLH = BH + 2;
constexpr int BLP = BLW * BLH;

template <int BC>
__device__ __forceinline__ int64_t map2(int64_t c, int64_t n)
{
    if (c >= 0 && c < n) return c;
    if (BC == BC_HN) return c < 0 ? 0 : n - 1;
    if (BC == BC_HD) return -1;
    const int64_t r = c % n;  // periodic: the ring may wrap more than once on tiny grids
    return r < 0 ? r + n : r;
}

// Global offset of region slot (y, x) BC-mapped, or -1 for the Dirichlet 0.
template <int BC>
__device__ __forceinline__ int64_t goff(const Shape &s, int64_t y, int64_t x)
{
    const int64_t my = map2<BC>(y, s.M1), mx = map2<BC>(x, s.M2);
    return (my < 0 || mx < 0) ? -1 : my * s.M2 + mx;
}

// Per-lane geometry of a region.
struct Geo {
    int64_t y0r, xg;  // global coordinates of region row 0 / this lane's column
    int K;
    int xm, xp;       // LDS column offsets of the x neighbours (BC-redirected)
};

// Geometry of region `tile` (tiles numbered row-major, tiles_x per row) for
// lane tx of a row.
template <int BC>
__device__ __forceinline__ Geo make_geo(const Shape &s, int K, int64_t tiles_x, int64_t tile, int tx)
{
    Geo g;
    const int oy = BH - 2 * K, ox = BX - 2 * K;
    g.y0r = (tile / tiles_x) * oy - K;
    g.xg = (tile % tiles_x) * ox - K + tx;
    g.K = K;
    g.xm = -1;
    g.xp = 1;
    if (BC != BC_P) {
        if (g.xg == 0) g.xm = (BC == BC_HN) ? 0 : -(tx + 1);          // own slot / pad column
        if (g.xg == s.M2 - 1) g.xp = (BC == BC_HN) ? 0 : (BX - tx);  // own slot / pad column
    }
    return g;
}

// LDS neighbour offsets of region row ry (BC-redirected in y).
template <int BC>
__device__ __forceinline__ void yoffs(const Shape &s, const Geo &g, int ry, int &ym, int &yp)
{
    ym = -BLW;
    yp = BLW;
    if (BC != BC_P) {
        const int64_t yg = g.y0r + ry;
        if (yg == 0) ym = (BC == BC_HN) ? 0 : -(ry + 1) * BLW;             // own slot / pad row 0
        if (yg == s.M1 - 1) yp = (BC == BC_HN) ? 0 : (BH - ry) * BLW;     // own slot / pad row
    }
}

}  // namespace tile2d
}  // namespace ace
