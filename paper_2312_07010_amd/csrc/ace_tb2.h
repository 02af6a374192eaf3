// 2D temporal blocking with the region held in registers: K steps of the
// scheme per launch (1 <= K <= the region's depth limit).
//
// A workgroup of TRW wavefronts loads the RH x 64 region (RH = TRW * RYT)
// around an (RH - 2K) x (64 - 2K) output tile, a ring of K nodes recomputed
// instead of exchanged.  Lane x of wavefront w holds the RYT consecutive
// region rows w RYT .. w RYT + RYT - 1 of column x in registers and advances
// them K times.  Per level the neighbours of a node are:
//   * along the row (i2): the neighbouring lanes' registers, moved by DPP
//     lane shifts (the lanes at the region's edge receive 0; they are ring
//     nodes, never needed at the next level);
//   * across rows (i1): the thread's own registers, except above its first
//     and below its last row, which come from the neighbouring wavefronts
//     through two LDS edge rows per wavefront, double-buffered by level
//     parity (one workgroup barrier per level).
// After level k only region rows k .. RH-1-k are still needed, so the rows
// outside are skipped (wave-uniform tests).
//
// Nodes outside the domain are loaded as the images the boundary condition
// makes of the field: periodic wraps; Neumann reflects about the wall half a
// cell past the last node (the ghost next to node 0 holds node 0, the next
// one node 1, ...); Dirichlet holds 0 at the wall node and the negated
// reflection beyond it.  The step maps these images to the images of the
// stepped field exactly: the update is odd in (node, neighbour sum) and the
// pair sums are commutative, so a mirrored ghost computes its node's value
// and a negated one its negative, bit for bit, and a Dirichlet wall node
// stays 0.  So every node, in the domain or not, takes its plain neighbours,
// and the boundary nodes get exactly the one-step kernels' values (Neumann:
// the outward neighbour is the node itself; Dirichlet: 0) with no test per
// node.  The arithmetic and the neighbour order are those of the one-step
// kernels, so the result equals K one-step launches bit for bit.  Monitors (MON) are those of the input
// field; LEVELS writes every level k to out + (k - 1) * level_stride (the
// adjoint's segment recompute).
#pragma once

#include "ace_device.h"

namespace ace {
namespace tb2 {

constexpr int RX = 64;  // region width: one wavefront

// Stored index of the node whose value (times *sign: +1, -1, or 0 for a
// Dirichlet wall node) the boundary condition places at coordinate c of an
// axis of n stored nodes (the ring may reach past the domain more than once
// on tiny grids).  Fields here have fewer than 2^31 nodes, so coordinates
// and offsets are 32-bit.
template <int BC>
__device__ __forceinline__ int image(int c, int n, int &sign)
{
    sign = 1;
    if (c >= 0 && c < n) return c;
    if (BC == BC_P) {
        const int r = c % n;
        return r < 0 ? r + n : r;
    }
    if (BC == BC_HN) {  // mirror about the walls at -1/2 and n - 1/2: period 2n
        int r = c % (2 * n);
        if (r < 0) r += 2 * n;
        return r < n ? r : 2 * n - 1 - r;
    }
    // Dirichlet: wall nodes at -1 and n (value 0), odd reflection about them:
    // period 2 (n + 1) in u = c + 1
    const int P = 2 * (n + 1);
    int u = (c + 1) % P;
    if (u < 0) u += P;
    if (u == 0 || u == n + 1) {
        sign = 0;
        return 0;
    }
    if (u <= n) return u - 1;
    sign = -1;
    return P - u - 1;
}

// The next lower lane's value (CTRL 0x138, DPP wave_shr:1) or the next higher
// lane's (0x130, wave_shl:1); lane 0 (resp. 63) receives 0.
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int TRW, int RYT>
struct Geom {
    static constexpr int NT = RX * TRW;
    static constexpr int RH = TRW * RYT;
    static constexpr int KMAX = RH / 2 - 4;  // keeps an (RH - 2 KMAX = 8) x (64 - 2 KMAX) tile
};

// One region of the blocked 2D step, shared by the kernel below (one region
// per workgroup) and the batched launch (each workgroup walks an instance's
// regions in turn).  EB is the workgroup's edge-row buffer of
// 2 * 2 * TRW * 64 doubles; `tile` numbers the (RH - 2K) x (64 - 2K) output
// tiles: tile row tile_y, column tile_x.  The field has fewer than 2^31
// nodes (32-bit offsets).
template <int BC, int TRW, int RYT>
struct Region {
    using G = Geom<TRW, RYT>;
    static constexpr int RH = G::RH;
    int K, tx, tr, M1, M2;
    int yr0, xg, mx;
    int sx;
    bool xin, xb0;

    __device__ __forceinline__ Region(const Shape &s, int K_, int tile_y, int tile_x) : K(K_)
    {
        M1 = (int)s.M1;
        M2 = (int)s.M2;
        tx = threadIdx.x & (RX - 1);
        tr = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront (uniform)
        const int oy = RH - 2 * K, ox = RX - 2 * K;
        yr0 = tile_y * oy - K;  // global row of region row 0
        xg = tile_x * ox - K + tx;
        mx = image<BC>(xg, M2, sx);
        xin = xg >= 0 && xg < M2 && tx >= K && tx < RX - K;
        xb0 = (xg == 0);
    }

    // level 0 of this thread's rows (images outside the domain)
    __device__ __forceinline__ void load(const Shape &s, const double *__restrict__ in, double (&v)[RYT]) const
    {
#pragma unroll
        for (int r = 0; r < RYT; ++r) {
            int sy;
            const int my = image<BC>(yr0 + tr * RYT + r, M1, sy);
            const int sg = sx * sy;
            const double val = in[my * M2 + mx];
            v[r] = (BC == BC_P || sg > 0) ? val : (sg < 0 ? -val : 0.0);
        }
    }

    // Advances v (level 0, loaded) K levels; MON accumulates the monitor
    // terms of level 0 over the tile interior into m; level K (LEVELS: every
    // level k at out + (k - 1) * level_stride) goes to the tile interior.
    // Ends with every wavefront past its last read of EB only if the caller
    // adds a barrier before EB is written again.
    template <bool MON, bool LEVELS, int RV>
    __device__ __forceinline__ void advance(const Shape &s, const StepCoef &c, double (&v)[RYT],
                                            double *__restrict__ out, int64_t level_stride, double *EB,
                                            MonAcc &m) const
    {
        auto eb = [&](int par, int side, int w) -> double * { return EB + ((par * 2 + side) * TRW + w) * RX; };
        // per row: the output offset of a tile-interior node in the domain (-1
        // otherwise; also the monitor's node set)
        int oof[RYT];
        bool yb0[RYT];
#pragma unroll
        for (int r = 0; r < RYT; ++r) {
            const int ry = tr * RYT + r;
            const int yg = yr0 + ry;
            oof[r] = (xin && ry >= K && ry < RH - K && yg >= 0 && yg < M1) ? yg * M2 + xg : -1;
            yb0[r] = (yg == 0);
        }
        eb(0, 0, tr)[tx] = v[0];
        eb(0, 1, tr)[tx] = v[RYT - 1];
        __syncthreads();
        // Level k from level k - 1.  FULL: every row of this wavefront is
        // computed at this level (no per-row test); STORE: the tile-interior
        // results go to out.
        auto level = [&](int k, auto FULLc, auto STOREc) __attribute__((always_inline)) {
            constexpr bool FULL = decltype(FULLc)::value, STORE = decltype(STOREc)::value;
            const int rd = (k - 1) & 1;
            // (region rows 0 and RH-1 are never computed, so wavefront 0
            // never uses eT nor wavefront TRW-1 eB: they read their own
            // edge rows instead, in bounds and unused)
            const double eT = eb(rd, 1, tr > 0 ? tr - 1 : 0)[tx];
            const double eB = eb(rd, 0, tr < TRW - 1 ? tr + 1 : TRW - 1)[tx];
            double *__restrict__ lout = out + (LEVELS ? (int64_t)(k - 1) * level_stride : 0);
            // (FULL with a compiled root variant: every row's xi first, then
            // all rows' roots together)
            constexpr bool JOINT = FULL && RV > 0;
            double nv[RYT], xi[RYT];
#pragma unroll
            for (int r = 0; r < RYT; ++r) {
                nv[r] = v[r];
                const int ry = tr * RYT + r;
                if (!FULL && (ry < k || ry >= RH - k)) continue;  // wave-uniform: a ring row of this level
                const double p = v[r];
                const double ym = (r > 0) ? v[r > 0 ? r - 1 : 0] : eT;
                const double yp = (r < RYT - 1) ? v[r < RYT - 1 ? r + 1 : 0] : eB;
                const double xm = lane_shift<0x138>(p);
                const double xp = lane_shift<0x130>(p);
                // (the monitor's nodes, the tile interior, are all level-1 rows)
                if (MON && k == 1 && oof[r] >= 0) {
                    // next-node differences with the BC value past the end (the
                    // image there), plus Dirichlet's first-node wall edge
                    const double dy = yp - p, dx = xp - p;
                    double gr = fma(dy, dy, dx * dx);
                    if (BC == BC_HD) {
                        if (yb0[r]) gr = fma(p, p, gr);
                        if (xb0) gr = fma(p, p, gr);
                    }
                    m.bulk += bulk_term(p);
                    m.grad += gr;
                    m.mx = nan_max(m.mx, fabs(p));
                }
                const double nsum = (ym + yp) + (xm + xp);
                if constexpr (JOINT) {
                    xi[r] = explicit_part<2>(p, nsum, c);
                } else {
                    const double val = update_n<2, RV>(p, nsum, c);
                    nv[r] = val;
                    if (STORE && oof[r] >= 0) lout[oof[r]] = val;
                }
            }
            if constexpr (JOINT) {
                cubic_roots_n<RV>(xi, nv, c);
#pragma unroll
                for (int r = 0; r < RYT; ++r)
                    if (STORE && oof[r] >= 0) lout[oof[r]] = nv[r];
            }
#pragma unroll
            for (int r = 0; r < RYT; ++r) v[r] = nv[r];
        };
        using T = std::true_type;
        using F = std::false_type;
        const int row0 = tr * RYT;
        for (int k = 1; k < K; ++k) {
            const bool full = row0 >= k && row0 + RYT <= RH - k;
            if (full) level(k, T(), std::integral_constant<bool, LEVELS>());
            else level(k, F(), std::integral_constant<bool, LEVELS>());
            eb(k & 1, 0, tr)[tx] = v[0];
            eb(k & 1, 1, tr)[tx] = v[RYT - 1];
            __syncthreads();
        }
        if (row0 >= K && row0 + RYT <= RH - K) level(K, T(), T());
        else level(K, F(), T());
    }
};

template <int BC, bool MON, bool LEVELS, int RV, int TRW, int RYT>
__global__ __launch_bounds__(RX * TRW) void k_tb2(Shape s, StepCoef c, const double *__restrict__ in,
                                                  double *__restrict__ out, double *__restrict__ partials,
                                                  int K, int tiles_x, int64_t level_stride)
{
    constexpr int NT = Geom<TRW, RYT>::NT;
    __shared__ double EB[2 * 2 * TRW * RX];  // [parity][top | bottom][wavefront][lane]
    __shared__ double red[3 * (NT / 64)];
    const int tile = (int)xcd_tile(blockIdx.x, gridDim.x);  // tiles numbered row-major
    const Region<BC, TRW, RYT> g(s, K, tile / tiles_x, tile - (tile / tiles_x) * tiles_x);
    double v[RYT];
    g.load(s, in, v);
    MonAcc m;
    mon_zero(m);
    g.template advance<MON, LEVELS, RV>(s, coef_vgpr(c), v, out, level_stride, EB, m);
    if (MON) block_reduce_store(m, red, partials + 3 * blockIdx.x);
}

template <int TRW, int RYT>
void tiles(const Shape &s, int K, int &tiles_x, int &ntiles)
{
    const int oy = Geom<TRW, RYT>::RH - 2 * K, ox = RX - 2 * K;
    tiles_x = (int)((s.M2 + ox - 1) / ox);
    ntiles = tiles_x * (int)((s.M1 + oy - 1) / oy);
}

// Dispatch over the boundary condition, the output mode (monitor partials,
// every level, last level) and the root variants.
template <int TRW, int RYT>
hipError_t launch_any(const Shape &s, const StepCoef &c, const double *in, double *out, double *partials,
                      int64_t *nparts, int K, int64_t level_stride, hipStream_t st)
{
    using G = Geom<TRW, RYT>;
    if (K < 1 || K > G::KMAX) return hipErrorInvalidValue;
    int tiles_x, ntiles;
    tiles<TRW, RYT>(s, K, tiles_x, ntiles);
    if (nparts) *nparts = ntiles;
    const bool levels = level_stride > 0;
    const int rv = root_variant(c);
    auto go = [&](auto BCc, auto RVc) {
        constexpr int B = decltype(BCc)::value, R = decltype(RVc)::value;
        if (partials)
            hipLaunchKernelGGL((k_tb2<B, true, false, R, TRW, RYT>), dim3(ntiles), dim3(G::NT), 0, st, s, c, in,
                               out, partials, K, tiles_x, level_stride);
        else if (levels)
            hipLaunchKernelGGL((k_tb2<B, false, true, R, TRW, RYT>), dim3(ntiles), dim3(G::NT), 0, st, s, c, in,
                               out, partials, K, tiles_x, level_stride);
        else
            hipLaunchKernelGGL((k_tb2<B, false, false, R, TRW, RYT>), dim3(ntiles), dim3(G::NT), 0, st, s, c,
                               in, out, partials, K, tiles_x, level_stride);
        return hipGetLastError();
    };
    auto by_rv = [&](auto BCc) {
        switch (rv) {
        case 1: return go(BCc, std::integral_constant<int, 1>());
        case 2: return go(BCc, std::integral_constant<int, 2>());
        case 3: return go(BCc, std::integral_constant<int, 3>());
        case 5: return go(BCc, std::integral_constant<int, 5>());
        case 6: return go(BCc, std::integral_constant<int, 6>());
        default: return go(BCc, std::integral_constant<int, 0>());
        }
    };
    switch (s.bc) {
    case BC_HN: return by_rv(std::integral_constant<int, BC_HN>());
    case BC_HD: return by_rv(std::integral_constant<int, BC_HD>());
    case BC_P: return by_rv(std::integral_constant<int, BC_P>());
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tb2
}  // namespace ace
