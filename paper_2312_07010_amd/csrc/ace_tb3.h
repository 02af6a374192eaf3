// 3D step kernel with temporal blocking of depth K (K time levels per HBM
// round trip) on configurable regions.
//
// A workgroup of TRW wavefronts owns an (RH - 2K) x (64 - 2K) output tile of
// the two fastest axes (i1, i2), RH = TRW * RYT, and a chunk of planes along
// i0.  It works on the RH x 64 region around the tile (a ring of K nodes,
// recomputed instead of exchanged) and marches along i0.  Lane x of
// wavefront w holds the RYT consecutive region rows w RYT .. w RYT + RYT - 1
// of column x in registers, for every time level, in register queues along
// i0 (level 0: planes zc-1 .. zc+1, the slot of zc-1 reloaded with plane
// zc+2 as soon as level 1 has read it, about two thirds of a position ahead
// of its use; level j = 1..K-1: the three planes that level j+1 needs
// next).  All queues have three slots, so three march positions fix every
// slot at compile time.  At march position zc it computes level j of plane
// zc - j + 1 for j = 1..K; level K is the output.  Of the seven neighbours of
// a node:
//   * i0: from the level's register queue;
//   * i1 within the thread's rows: registers; across wavefronts (the top and
//     bottom rows of each wavefront's block): LDS edge buffers, one pair per
//     level and march parity (published at position zc, read at zc + 1,
//     with one workgroup barrier per position);
//   * i2: the neighbouring lanes' registers, moved by DPP lane shifts (no LDS
//     round trip on the critical path; the lane at the region edge receives
//     0, a ring node).
// The LDS holds per level only two rows per wavefront.  Every value that
// reaches the output is computed with exactly the arithmetic and neighbour
// order of the one-step kernels, so K steps of this kernel equal K one-step
// launches bit for bit.
//
// Boundary conditions.  Level-0 values outside the domain are loaded
// BC-mapped (clamped node for Neumann, 0 for Dirichlet, wrapped node for
// periodic), so level 1 is right at every in-domain node and, for periodic,
// also at the ring nodes.  For Neumann and Dirichlet a boundary node's
// outward neighbour at level >= 1 is the node itself (mirror) or 0 instead of
// the (inexact) ring value.
#pragma once

#include "ace_device.h"

namespace ace {
namespace tb3 {

constexpr int RX = 64;  // region width: one wavefront

// Coordinate c on an axis of n nodes, BC-mapped: Neumann clamps, Dirichlet
// returns -1 (the zero wall), periodic wraps (possibly more than once).
template <int BC>
__device__ __forceinline__ int64_t mapc(int64_t c, int64_t n)
{
    if (c >= 0 && c < n) return c;
    if (BC == BC_HN) return c < 0 ? 0 : n - 1;
    if (BC == BC_HD) return -1;
    const int64_t r = c % n;
    return r < 0 ? r + n : r;
}

// Raw buffer resources over one plane: the fourth descriptor word of
// the gfx9 family, and a byte offset past any plane (2^31, with planes
// below 2^31 bytes), at which a store falls outside the buffer and is
// dropped by the hardware's range check instead of an execution mask.
constexpr int kBufWord3 = 0x00020000;
constexpr uint32_t kNoStore = 0x80000000u;
using BufB64 = decltype(__builtin_amdgcn_raw_buffer_load_b64(__amdgpu_buffer_rsrc_t(), 0, 0, 0));

// mapc of a plane index that advances one plane at a time, with its element
// offset (mapped index times the plane size; -1 for the Dirichlet zero
// plane), kept up to date by comparisons instead of a division and a product
// per plane.
template <int BC>
struct PlaneCursor {
    int64_t z, mz, off;
    __device__ __forceinline__ void init(int64_t z0, int64_t n, int64_t PS)
    {
        z = z0;
        mz = mapc<BC>(z0, n);
        off = mz < 0 ? -1 : mz * PS;
    }
    __device__ __forceinline__ void next(int64_t n, int64_t PS)
    {
        ++z;
        if (BC == BC_P) {  // (mz + 1) mod n
            ++mz;
            off += PS;
            if (mz == n) {
                mz = 0;
                off = 0;
            }
        } else if (z <= 0) {  // below the domain (Neumann: node 0) or its first plane
            mz = (BC == BC_HN || z == 0) ? 0 : -1;
            off = (BC == BC_HN || z == 0) ? 0 : -1;
        } else if (z < n) {  // the previous plane was z - 1, in the domain
            mz = z;
            off += PS;
        } else if (BC == BC_HD) {  // past the domain: the zero wall
            mz = -1;
            off = -1;
        }  // (Neumann past the domain: stays at node n - 1)
    }
};

// The value of the next lower lane (CTRL = 0x138, DPP wave_shr:1) or the next
// higher lane (CTRL = 0x130, wave_shl:1) of a 64-lane wavefront, moved
// between registers by the DPP lane network in two 32-bit halves; lane 0
// (resp. 63) receives 0.
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int K, int TRW, int RYT>
struct Geom {
    static constexpr int NT = RX * TRW;      // threads
    static constexpr int RH = TRW * RYT;     // region rows
    static constexpr int OX = RX - 2 * K;    // output tile width
    static constexpr int OY = RH - 2 * K;    // output tile height
    static constexpr int NQ = K > 1 ? K - 1 : 1;  // level queues 1..K-1
    static_assert(OY >= 4, "region too short for the depth");
};

template <int BC, bool MON, int RV, int K, int TRW, int RYT, int OCC>
__global__ __launch_bounds__(RX * TRW) __attribute__((amdgpu_waves_per_eu(OCC))) void k_tb3(
    Shape s, StepCoef c0, const double *__restrict__ in, double *__restrict__ out,
    double *__restrict__ partials, int tiles_x, int tiles_y, int zchunk)
{
    using G = Geom<K, TRW, RYT>;
    const StepCoef c = coef_vgpr(c0);
    constexpr int NT = G::NT, RH = G::RH, OX = G::OX, OY = G::OY;
    __shared__ double EB[K * 2 * 2 * TRW * RX];  // [level][parity][top|bottom][wavefront][lane]
    __shared__ double red[3 * (NT / 64)];

    const int tx = threadIdx.x & (RX - 1);
    const int tr = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront index (uniform)
    auto eb = [&](int lvl, int par, int side, int w) -> double * {
        return EB + (((lvl * 2 + par) * 2 + side) * TRW + w) * RX;
    };

    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);  // XCD-aware numbering
    const int64_t ntile = (int64_t)tiles_x * tiles_y;
    int64_t lo, hi;
    if (zchunk > 0) {
        const int64_t tile = t % ntile, chunk = t / ntile;
        lo = tile * s.M0 + chunk * zchunk;
        hi = tile * s.M0 + ((chunk + 1) * zchunk < s.M0 ? (chunk + 1) * zchunk : s.M0);
    } else {
        const int64_t P = ntile * s.M0;
        lo = t * P / gridDim.x;
        hi = (t + 1) * P / gridDim.x;
    }
    const int64_t PS = s.M1 * s.M2;
    MonAcc m;
    mon_zero(m);

    while (lo < hi) {
        const int64_t tile_xy = lo / s.M0;
        const int64_t z0 = lo - tile_xy * s.M0;
        const int64_t z1 = (z0 + (hi - lo) < s.M0) ? z0 + (hi - lo) : s.M0;
        lo += z1 - z0;
        const int tile_x = (int)(tile_xy % tiles_x);
        const int tile_y = (int)(tile_xy / tiles_x);
        const int64_t yr0 = (int64_t)tile_y * OY - K;  // global row of region row 0
        const int64_t xg = (int64_t)tile_x * OX - K + tx;
        const int64_t mxc = mapc<BC>(xg, s.M2);
        const bool xb0 = (xg == 0), xb1 = (xg == s.M2 - 1);

        // per row: mapped in-plane load offset in bytes (-1: Dirichlet zero),
        // output offset in bytes (kNoStore: ring or outside the domain),
        // domain-edge flags (uniform)
        int off[RYT];
        uint32_t oof[RYT];
        bool yb0[RYT], yb1[RYT];
#pragma unroll
        for (int r = 0; r < RYT; ++r) {
            const int ry = tr * RYT + r;
            const int64_t yg = yr0 + ry;
            const int64_t myc = mapc<BC>(yg, s.M1);
            off[r] = (myc < 0 || mxc < 0) ? -1 : (int)(myc * s.M2 + mxc) * 8;
            const bool interior = ry >= K && ry < RH - K && tx >= K && tx < RX - K;
            const bool indomain = yg >= 0 && yg < s.M1 && xg >= 0 && xg < s.M2;
            oof[r] = (interior && indomain) ? (uint32_t)(yg * s.M2 + xg) * 8u : kNoStore;
            yb0[r] = (yg == 0);
            yb1[r] = (yg == s.M1 - 1);
        }
        auto base = [&](int64_t z) -> int64_t {
            const int64_t mz = mapc<BC>(z, s.M0);
            return mz < 0 ? -1 : mz * PS;
        };
        // (a buffer over the input plane and a 32-bit byte offset per lane)
        auto ld = [&](int64_t b, int o) -> double {
            auto at = [&]() {
                const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<double *>(in) + (b < 0 ? 0 : b), (short)0, (int)(PS * 8), kBufWord3);
                return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0));
            };
            if (BC != BC_HD) return at();
            return (b < 0 || o < 0) ? 0.0 : at();
        };

        // level-0 queue: slot k holds plane zs - 1 + k at the first position
        const int64_t zs = z0 - K + 1;           // first march position
        const int64_t zend = z1 + K - 2;         // last march position
        const int64_t zlast = z1 + K - 1;        // last level-0 plane needed
        double q0[3][RYT];
        double qj[G::NQ][3][RYT];
        {
            const int64_t b0 = base(zs - 1), b1 = base(zs), b2 = base(zs + 1);
#pragma unroll
            for (int r = 0; r < RYT; ++r) {
                q0[0][r] = ld(b0, off[r]);
                q0[1][r] = ld(b1, off[r]);
                q0[2][r] = ld(b2, off[r]);
            }
        }
#pragma unroll
        for (int j = 0; j < G::NQ; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int r = 0; r < RYT; ++r) qj[j][k][r] = 0.0;
        // the plane the next position loads, and the output offset of plane
        // zc - K + 1 (level K's plane)
        static_assert(K >= 2, "the cursor starts at the last plane loaded above");
        PlaneCursor<BC> cur;
        cur.init(zs + 1, s.M0, PS);
        int64_t ooff = (zs - K + 1) * PS;
        // edges of level-0 plane zs, read at the first position
        eb(0, (int)((zs - 1) & 1), 0, tr)[tx] = q0[1][0];
        eb(0, (int)((zs - 1) & 1), 1, tr)[tx] = q0[1][RYT - 1];
        __syncthreads();

        int64_t zc = zs;

        // Level J (1..K) of plane zo = zc - J + 1 from level J-1: zm, cq, zp
        // are the level J-1 values of planes zo-1, zo, zo+1; the result goes
        // to dst (J < K) or to the output (J == K).
        auto level = [&](auto JJ, const double(&zmq)[RYT], const double(&cq)[RYT],
                         const double(&zpq)[RYT], double(&dst)[RYT]) __attribute__((always_inline)) {
            constexpr int J = decltype(JJ)::value;
            const int64_t zo = zc - J + 1;
            const int rd = (int)((zc - 1) & 1);
            // i2 neighbours: the neighbouring lanes' values of the same row
            double xm[RYT], xp[RYT];
#pragma unroll
            for (int r = 0; r < RYT; ++r) {
                xm[r] = lane_shift<0x138>(cq[r]);
                xp[r] = lane_shift<0x130>(cq[r]);
            }
            // i1 neighbours across wavefronts.  Wavefront 0's eT and wavefront
            // TRW-1's eB would lie outside the region: they read their own
            // edge rows instead (in bounds, no branch).  The rows they feed,
            // region rows 0 and RH-1, are ring rows at every level.
            const double eT = eb(J - 1, rd, 1, tr > 0 ? tr - 1 : 0)[tx];
            const double eB = eb(J - 1, rd, 0, tr < TRW - 1 ? tr + 1 : TRW - 1)[tx];
            const bool mon_plane = MON && J == 1 && zo >= z0 && zo < z1;
            // buffer over output plane zo (used at J == K only): rows at
            // offset kNoStore fall outside it and are not written
            const __amdgpu_buffer_rsrc_t orsrc =
                __builtin_amdgcn_make_buffer_rsrc(out + (J == K ? ooff : 0), (short)0, (int)(PS * 8), kBufWord3);
            // Every row is computed, also the ring rows ry < J and
            // ry >= RH - J, whose values at this level are wrong: they only
            // reach ring rows of the next level and rows that are neither
            // stored nor monitored (oof is kNoStore there), and skipping them
            // would cost a test per row in every wavefront to spare work in
            // the two edge wavefronts, which otherwise wait at the barrier.
            double xi[RYT], th[RYT];  // (compiled root variants: all rows' roots at once)
#pragma unroll
            for (int r = 0; r < RYT; ++r) {
                const double p = cq[r];
                double zm = zmq[r], zp = zpq[r];
                double ym = (r > 0) ? cq[r > 0 ? r - 1 : 0] : eT;
                double yp = (r < RYT - 1) ? cq[r < RYT - 1 ? r + 1 : 0] : eB;
                double xmv = xm[r], xpv = xp[r];
                if (BC != BC_P && J >= 2) {
                    const double wall = (BC == BC_HN) ? p : 0.0;
                    if (zo == 0) zm = wall;
                    if (zo == s.M0 - 1) zp = wall;
                    if (yb0[r]) ym = wall;
                    if (yb1[r]) yp = wall;
                    if (xb0) xmv = wall;
                    if (xb1) xpv = wall;
                }
                const double nsum = ((zm + zp) + (ym + yp)) + (xmv + xpv);
                if constexpr (RV > 0) {
                    xi[r] = explicit_part<3>(p, nsum, c);
                } else {
                    const double v = update_n<3, RV>(p, nsum, c);
                    if (J < K) dst[r] = v;
                    else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufB64, v), orsrc, (int)oof[r], 0, 0);
                }
                if (mon_plane && oof[r] != kNoStore) {
                    const double dz = zp - p, dy = yp - p, dx = xpv - p;
                    double g = fma(dz, dz, fma(dy, dy, dx * dx));
                    if (BC == BC_HD) {
                        if (zo == 0) g = fma(p, p, g);
                        if (yb0[r]) g = fma(p, p, g);
                        if (xb0) g = fma(p, p, g);
                    }
                    m.bulk += bulk_term(p);
                    m.grad += g;
                    m.mx = nan_max(m.mx, fabs(p));
                }
            }
            if constexpr (RV > 0) {
                cubic_roots_n<RV>(xi, th, c);
#pragma unroll
                for (int r = 0; r < RYT; ++r) {
                    if (J < K) dst[r] = th[r];
                    else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufB64, th[r]), orsrc, (int)oof[r], 0, 0);
                }
            }
            if (J < K) {
                const int wr = (int)(zc & 1);
                eb(J, wr, 0, tr)[tx] = dst[0];
                eb(J, wr, 1, tr)[tx] = dst[RYT - 1];
            }
        };

        // One march position with the queue slots fixed at compile time:
        // level 0 planes zc-1, zc, zc+1 in q0[S % 3 ..], level j planes
        // zc-j-1, zc-j, zc-j+1 in qj[j-1][S % 3 ..] (the last written here).
        auto body = [&](auto SS) __attribute__((always_inline)) -> bool {
            constexpr int S = decltype(SS)::value;
            constexpr int P0 = S % 3, P1 = (S + 1) % 3, P2 = (S + 2) % 3;
            // level 1 of plane zc
            level(std::integral_constant<int, 1>(), q0[P0], q0[P1], q0[P2], qj[0][P2]);
            // next level-0 plane into the slot level 1 just freed
            {
                if (zc + 2 <= zlast) cur.next(s.M0, PS);  // plane min(zc + 2, zlast)
                const int64_t bn = cur.off;
#pragma unroll
                for (int r = 0; r < RYT; ++r) q0[P0][r] = ld(bn, off[r]);
            }
            // levels 2..K, each from the one below (active once its inputs exist)
            if constexpr (K >= 2) {
                if (zc >= z0 - K + 3)
                    level(std::integral_constant<int, 2>(), qj[0][P0], qj[0][P1], qj[0][P2],
                          qj[K >= 3 ? 1 : 0][P2]);
            }
            if constexpr (K >= 3) {
                if (zc >= z0 - K + 5)
                    level(std::integral_constant<int, 3>(), qj[1][P0], qj[1][P1], qj[1][P2],
                          qj[K >= 4 ? 2 : 1][P2]);
            }
            if constexpr (K >= 4) {
                if (zc >= z0 - K + 7)
                    level(std::integral_constant<int, 4>(), qj[2][P0], qj[2][P1], qj[2][P2], qj[2][P2]);
            }
            if (zc >= zend) return true;
            // edges of level-0 plane zc+1 for the next position
            eb(0, (int)(zc & 1), 0, tr)[tx] = q0[P2][0];
            eb(0, (int)(zc & 1), 1, tr)[tx] = q0[P2][RYT - 1];
            __syncthreads();
            ++zc;
            ooff += PS;
            return false;
        };
        for (;;) {
            if (body(std::integral_constant<int, 0>())) break;
            if (body(std::integral_constant<int, 1>())) break;
            if (body(std::integral_constant<int, 2>())) break;
        }
        __syncthreads();  // every wavefront is done with the edge buffers of this segment
    }
    if (MON) block_reduce_store(m, red, partials + 3 * t);
}

}  // namespace tb3
}  // namespace ace

namespace ace {
namespace tb3 {

// Tile counts of a region shape on the (i1, i2) plane.
template <int K, int TRW, int RYT>
void tiles(const Shape &s, int &tiles_x, int &tiles_y)
{
    using G = Geom<K, TRW, RYT>;
    tiles_x = (int)((s.M2 + G::OX - 1) / G::OX);
    tiles_y = (int)((s.M1 + G::OY - 1) / G::OY);
}

constexpr int64_t PERSIST_MIN = 16;  // least tile-planes per persistent workgroup

template <int K, int TRW, int RYT>
int64_t partials_needed(const Shape &s, int zchunk)
{
    int tx, ty;
    tiles<K, TRW, RYT>(s, tx, ty);
    const int64_t nt = (int64_t)tx * ty;
    if (zchunk <= 0) return std::max<int64_t>(1, std::min<int64_t>(8192, nt * s.M0 / PERSIST_MIN));
    return nt * ((s.M0 + zchunk - 1) / zchunk);
}

// Workgroups of one kernel instance that fit on the device at once (cached
// per device; 0 if the query fails).
template <int BC, bool MON, int RV, int K, int TRW, int RYT, int OCC>
int64_t resident_blocks()
{
    static int64_t cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cache[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tb3<BC, MON, RV, K, TRW, RYT, OCC>,
                                                         RX * TRW, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cache[dev] = (int64_t)std::max(per_cu, 1) * cus;
    }
    return cache[dev];
}

template <int BC, bool MON, int RV, int K, int TRW, int RYT, int OCC>
hipError_t launch(const Shape &s, const StepCoef &c, const double *in, double *out, double *partials,
                  int64_t *nparts, int zchunk, hipStream_t st)
{
    int tiles_x, tiles_y;
    tiles<K, TRW, RYT>(s, tiles_x, tiles_y);
    int64_t nblk;
    if (zchunk > 0) {
        nblk = (int64_t)tiles_x * tiles_y * ((s.M0 + zchunk - 1) / zchunk);
    } else {
        const int64_t res = resident_blocks<BC, MON, RV, K, TRW, RYT, OCC>();
        if (res <= 0) return hipErrorInvalidValue;
        nblk = std::min<int64_t>(res, partials_needed<K, TRW, RYT>(s, 0));
    }
    if (nblk < 1 || nblk > INT32_MAX) return hipErrorInvalidValue;
    if (nparts) *nparts = nblk;
    hipLaunchKernelGGL((k_tb3<BC, MON, RV, K, TRW, RYT, OCC>), dim3((unsigned)nblk), dim3(RX * TRW), 0, st,
                       s, c, in, out, partials, tiles_x, tiles_y, zchunk);
    return hipGetLastError();
}

// Dispatch over the boundary condition, the monitor flag and the root
// variants instantiated for this kernel (1: one Newton step, the benchmark's
// time step; 0: start and step count from the coefficients at run time,
// with the same rounding).
template <int K, int TRW, int RYT, int OCC>
hipError_t launch_any(const Shape &s, const StepCoef &c, const double *in, double *out,
                      double *partials, int64_t *nparts, int zchunk, hipStream_t st)
{
    const int rv = root_variant(c);
    auto go = [&](auto BCc, auto RVc) {
        constexpr int B = decltype(BCc)::value, R = decltype(RVc)::value;
        return partials ? launch<B, true, R, K, TRW, RYT, OCC>(s, c, in, out, partials, nparts, zchunk, st)
                        : launch<B, false, R, K, TRW, RYT, OCC>(s, c, in, out, partials, nparts, zchunk, st);
    };
    auto by_rv = [&](auto BCc) {
        switch (rv) {
        case 1: return go(BCc, std::integral_constant<int, 1>());
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

}  // namespace tb3
}  // namespace ace
