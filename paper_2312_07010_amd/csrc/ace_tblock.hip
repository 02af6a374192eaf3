// 3D step kernel with temporal blocking: two time levels per HBM round trip.
//
// A workgroup owns a 28 x 60 output tile of the two fastest axes (i1, i2) and
// a chunk of planes along i0.  It works on the 32 x 64 region around the tile
// (a ring of two nodes) and marches along i0.  At each position zc of the
// march it
//   A. computes level 1 (phi^{n+1}) of plane zc on the whole region from
//      level 0 (phi^n): i1/i2 neighbours from the level-0 plane in LDS, i0
//      neighbours from a per-thread register queue;
//   C. computes level 2 (phi^{n+2}) of plane zc-1 on the tile from level 1:
//      i1/i2 neighbours from the previous level-1 plane in LDS, i0 neighbours
//      from a level-1 register queue, and writes it to HBM;
//   D. stages level-0 plane zc+1 into the other LDS buffer (one barrier per
//      plane; both levels are double-buffered).
// Every value is computed with exactly the arithmetic and neighbour order of
// the one-step kernels, so two steps of this kernel equal two one-step
// launches bit for bit; the ring is recomputed redundantly instead of being
// exchanged between workgroups.
//
// Boundary conditions.  Level-0 slots outside the domain hold the value the
// BC assigns (clamped node for Neumann, 0 for Dirichlet, wrapped node for
// periodic), so level 1 is right at every in-domain slot, and for periodic
// also at the ring slots (they are wrapped nodes).  For Neumann and Dirichlet
// the level-2 update of a boundary node reads its outward neighbour from its
// own slot (mirror) or from a zero pad instead of from the ring.
#include "ace_device.h"

namespace ace {

namespace {

constexpr int RX = 64;           // region width: one wavefront
constexpr int TRW = 8;           // thread rows
constexpr int RYT = 4;           // region rows per thread
constexpr int RH = TRW * RYT;    // region height 32
constexpr int OX = RX - 4;       // tile (output) width 60
constexpr int OY = RH - 4;       // tile height 28
constexpr int NT = RX * TRW;     // 512 threads
constexpr int LW = RX + 2;       // LDS plane with a zero pad all around
constexpr int LH = RH + 2;
constexpr int LP = LW * LH;
constexpr int64_t PERSIST_MIN = 16;  // least tile-planes per persistent workgroup

template <int BC>
__device__ __forceinline__ int64_t map_coord2(int64_t c, int64_t n)
{
    if (c >= 0 && c < n) return c;
    if (BC == BC_HN) return c < 0 ? 0 : n - 1;
    if (BC == BC_HD) return -1;
    if (c < 0) return c + n >= 0 ? c + n : n - 1;
    return c - n < n ? c - n : 0;
}

template <int BC>
__device__ __forceinline__ int64_t plane_offset2(const Shape &s, int64_t y, int64_t x)
{
    const int64_t my = map_coord2<BC>(y, s.M1);
    const int64_t mx = map_coord2<BC>(x, s.M2);
    if (my < 0 || mx < 0) return -1;
    return my * s.M2 + mx;
}

template <int BC>
__device__ __forceinline__ int64_t plane_base2(const Shape &s, int64_t z)
{
    const int64_t mz = map_coord2<BC>(z, s.M0);
    return mz < 0 ? -1 : mz * s.M1 * s.M2;
}

// Mapped plane bases and row offsets are never negative for Neumann and
// periodic, so those loads are unconditional (no exec-masked branches in the
// march); Dirichlet marks the zero nodes outside the domain with -1.
template <int BC>
__device__ __forceinline__ double load_at2(const double *__restrict__ in, int64_t base, int64_t off)
{
    if (BC != BC_HD) return in[base + off];
    return (base < 0 || off < 0) ? 0.0 : in[base + off];
}

// amdgpu_waves_per_eu(4) caps the kernel at 128 VGPRs, so two 512-thread
// workgroups (LDS 72 KB each) share a CU.
template <int BC, bool MON, int RV>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_tblock3d(
    Shape s, StepCoef c, const double *__restrict__ in, double *__restrict__ out,
    double *__restrict__ partials, int tiles_x, int tiles_y, int zchunk)
{
    __shared__ double L0[2 * LP];
    __shared__ double L1[2 * LP];
    __shared__ double red[3 * (NT / 64)];

    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);  // XCD-aware numbering
    const int64_t ntile = (int64_t)tiles_x * tiles_y;
    // The workgroup's share of the tile-planes, numbered tile-major
    // (tile * M0 + plane): one chunk of one tile, or (zchunk = 0, a
    // persistent grid) an even share of all of them, which it marches as one
    // segment per tile it touches.
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
    const int tx = threadIdx.x & (RX - 1);
    const int tr = threadIdx.x / RX;
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
    const int64_t yr0 = (int64_t)tile_y * OY - 2;  // global row of region row 0
    const int64_t xg = (int64_t)tile_x * OX - 2 + tx;

    for (int i = threadIdx.x; i < 2 * LP; i += NT) {
        L0[i] = 0.0;
        L1[i] = 0.0;
    }

    // per-row slot data: global load offset, own LDS slot, level-2 neighbour
    // slots (BC-redirected), output offset (or -1)
    int64_t off[RYT], oof[RYT];
    int own[RYT], nym[RYT], nyp[RYT], nxm[RYT], nxp[RYT];
    bool edge_x0 = false, edge_y0[RYT];
#pragma unroll
    for (int r = 0; r < RYT; ++r) {
        const int ry = tr * RYT + r;
        const int64_t yg = yr0 + ry;
        off[r] = plane_offset2<BC>(s, yg, xg);
        own[r] = (ry + 1) * LW + (tx + 1);
        nym[r] = own[r] - LW;
        nyp[r] = own[r] + LW;
        nxm[r] = own[r] - 1;
        nxp[r] = own[r] + 1;
        if (BC != BC_P) {
            if (yg == 0) nym[r] = (BC == BC_HN) ? own[r] : (tx + 1);
            if (yg == s.M1 - 1) nyp[r] = (BC == BC_HN) ? own[r] : (LH - 1) * LW + (tx + 1);
            if (xg == 0) nxm[r] = (BC == BC_HN) ? own[r] : (ry + 1) * LW;
            if (xg == s.M2 - 1) nxp[r] = (BC == BC_HN) ? own[r] : (ry + 1) * LW + (LW - 1);
        }
        const bool interior = ry >= 2 && ry < RH - 2 && tx >= 2 && tx < RX - 2;
        const bool indomain = yg >= 0 && yg < s.M1 && xg >= 0 && xg < s.M2;
        oof[r] = (interior && indomain) ? yg * s.M2 + xg : -1;
        edge_y0[r] = (yg == 0);
    }
    edge_x0 = (xg == 0);

    // level-0 queue: q0 = plane zc-1, q1 = zc, q2 = zc+1, q3 = zc+2
    double q0[RYT], q1[RYT], q2[RYT], q3[RYT];
    {
        const int64_t bA = plane_base2<BC>(s, z0 - 2), bB = plane_base2<BC>(s, z0 - 1);
        const int64_t bC = plane_base2<BC>(s, z0), bD = plane_base2<BC>(s, z0 + 1);
#pragma unroll
        for (int r = 0; r < RYT; ++r) {
            q0[r] = load_at2<BC>(in, bA, off[r]);
            q1[r] = load_at2<BC>(in, bB, off[r]);
            q2[r] = load_at2<BC>(in, bC, off[r]);
            q3[r] = load_at2<BC>(in, bD, off[r]);
        }
    }
    __syncthreads();  // zero pads written before the first staging
#pragma unroll
    for (int r = 0; r < RYT; ++r) L0[own[r]] = q1[r];
    __syncthreads();

    // level-1 queue (plane zc-2, zc-1, zc) and the march.  The body below is
    // written once against named queue slots; the loop calls it with the
    // slots rotated (period 4 for level 0, 3 for level 1, so 12 calls per
    // turn), which replaces the queue shifts by register renaming.
    double w0[RYT], w1[RYT], w2[RYT];
#pragma unroll
    for (int r = 0; r < RYT; ++r) {
        w0[r] = 0.0;
        w1[r] = 0.0;
        w2[r] = 0.0;
    }
    int bl0 = 0, bl1 = 0;
    int64_t zc = z0 - 1;
    // rows a wavefront can skip: level 1 is needed on region rows 1..RH-2,
    // level 2 on the tile rows 2..RH-3 (a wavefront is one thread row, so
    // these tests are uniform across it)
    auto need1 = [&](int r) { const int ry = tr * RYT + r; return ry >= 1 && ry < RH - 1; };
    auto need2 = [&](int r) { const int ry = tr * RYT + r; return ry >= 2 && ry < RH - 2; };

    auto body = [&](double(&Q0)[RYT], double(&Q1)[RYT], double(&Q2)[RYT], double(&Q3)[RYT],
                    double(&W0)[RYT], double(&W1)[RYT], double(&W2)[RYT]) __attribute__((always_inline)) {
        // Q0..Q3: level-0 planes zc-1..zc+2; W0, W1: level-1 planes zc-2, zc-1
        const double *l0 = L0 + bl0 * LP;
        double *l1w = L1 + bl1 * LP;
        const double *l1r = L1 + (bl1 ^ 1) * LP;
        // --- A: level 1 of plane zc on the region ---
        const bool mon_plane = MON && zc >= z0 && zc < z1;
#pragma unroll
        for (int r = 0; r < RYT; ++r) {
            if (!need1(r)) continue;
            const double p = Q1[r];
            const double xm = l0[own[r] - 1];
            const double xp = l0[own[r] + 1];
            const double ym = (r > 0) ? Q1[r > 0 ? r - 1 : 0] : l0[own[r] - LW];
            const double yp = (r < RYT - 1) ? Q1[r < RYT - 1 ? r + 1 : 0] : l0[own[r] + LW];
            const double nsum = ((Q0[r] + Q2[r]) + (ym + yp)) + (xm + xp);
            const double v = update_n<3, RV>(p, nsum, c);
            W2[r] = v;
            l1w[own[r]] = v;
            if (mon_plane && oof[r] >= 0) {
                const double dz = Q2[r] - p, dy = yp - p, dx = xp - p;
                double g = fma(dz, dz, fma(dy, dy, dx * dx));
                if (BC == BC_HD) {
                    if (zc == 0) g = fma(p, p, g);
                    if (edge_y0[r]) g = fma(p, p, g);
                    if (edge_x0) g = fma(p, p, g);
                }
                m.bulk += bulk_term(p);
                m.grad += g;
                m.mx = nan_max(m.mx, fabs(p));
            }
        }
        // --- B: next level-0 plane zc+3 into the slot A just freed (Q0).  Issued
        // before C's stores so the loads have C, the staging and the barrier
        // to arrive in.  Past the last plane the segment needs (z1+1) the
        // load repeats that plane (unused). ---
        {
            const int64_t bn = plane_base2<BC>(s, (zc + 3 <= z1 + 1) ? zc + 3 : z1 + 1);
#pragma unroll
            for (int r = 0; r < RYT; ++r) Q0[r] = load_at2<BC>(in, bn, off[r]);
        }
        // --- C: level 2 of plane zc-1 on the tile ---
        if (zc >= z0 + 1) {
            const int64_t zo = zc - 1;
            double *const orow = out + zo * PS;
#pragma unroll
            for (int r = 0; r < RYT; ++r) {
                if (!need2(r)) continue;
                const double p = W1[r];
                double zm = W0[r], zp = W2[r];
                if (BC != BC_P) {
                    if (zo == 0) zm = (BC == BC_HN) ? p : 0.0;
                    if (zo == s.M0 - 1) zp = (BC == BC_HN) ? p : 0.0;
                }
                const double xm = l1r[nxm[r]];
                const double xp = l1r[nxp[r]];
                const double ym = l1r[nym[r]];
                const double yp = l1r[nyp[r]];
                const double nsum = ((zm + zp) + (ym + yp)) + (xm + xp);
                const double v = update_n<3, RV>(p, nsum, c);
                if (oof[r] >= 0) orow[oof[r]] = v;
            }
        }
        if (zc >= z1) return true;
        // --- stage plane zc+1 ---
        bl0 ^= 1;
        bl1 ^= 1;
#pragma unroll
        for (int r = 0; r < RYT; ++r) L0[bl0 * LP + own[r]] = Q2[r];
        __syncthreads();
        ++zc;
        return false;
    };
    double(&qa)[RYT] = q0;
    double(&qb)[RYT] = q1;
    double(&qc)[RYT] = q2;
    double(&qd)[RYT] = q3;
    for (;;) {
        if (body(qa, qb, qc, qd, w0, w1, w2)) break;
        if (body(qb, qc, qd, qa, w1, w2, w0)) break;
        if (body(qc, qd, qa, qb, w2, w0, w1)) break;
        if (body(qd, qa, qb, qc, w0, w1, w2)) break;
        if (body(qa, qb, qc, qd, w1, w2, w0)) break;
        if (body(qb, qc, qd, qa, w2, w0, w1)) break;
        if (body(qc, qd, qa, qb, w0, w1, w2)) break;
        if (body(qd, qa, qb, qc, w1, w2, w0)) break;
        if (body(qa, qb, qc, qd, w2, w0, w1)) break;
        if (body(qb, qc, qd, qa, w0, w1, w2)) break;
        if (body(qc, qd, qa, qb, w1, w2, w0)) break;
        if (body(qd, qa, qb, qc, w2, w0, w1)) break;
    }
    __syncthreads();  // every wavefront is done with the LDS planes of this segment
    }
    if (MON) block_reduce_store(m, red, partials + 3 * t);
}

}  // namespace

bool tblock_supported(const Shape &s)
{
    return s.d == 3 && s.M0 >= 1 && s.M1 >= 1 && s.M2 >= 1;
}

int64_t tblock_partials_needed(const Shape &s, int zchunk)
{
    const int64_t tiles = ((s.M2 + OX - 1) / OX) * ((s.M1 + OY - 1) / OY);
    if (zchunk <= 0) return std::max<int64_t>(1, std::min<int64_t>(8192, tiles * s.M0 / PERSIST_MIN));
    return tiles * ((s.M0 + zchunk - 1) / zchunk);
}

namespace {

// Workgroups of one kernel instance that fit on the device at once (cached
// per device and instance; 0 if the query fails).
template <int BC, bool MON, int RV>
int64_t resident_blocks()
{
    static int64_t cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cache[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tblock3d<BC, MON, RV>, NT, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cache[dev] = (int64_t)std::max(per_cu, 1) * cus;
    }
    return cache[dev];
}

template <int BC, bool MON, int RV>
hipError_t launch_tb(const Shape &s, const StepCoef &c, const double *in, double *out,
                     double *partials, int64_t *nparts, int zchunk, hipStream_t st)
{
    const int tiles_x = (int)((s.M2 + OX - 1) / OX);
    const int tiles_y = (int)((s.M1 + OY - 1) / OY);
    int64_t nblk;
    if (zchunk > 0) {
        nblk = (int64_t)tiles_x * tiles_y * ((s.M0 + zchunk - 1) / zchunk);
    } else {
        const int64_t res = resident_blocks<BC, MON, RV>();
        if (res <= 0) return hipErrorInvalidValue;
        nblk = std::min<int64_t>(res, tblock_partials_needed(s, 0));
    }
    if (nparts) *nparts = nblk;
    hipLaunchKernelGGL((k_tblock3d<BC, MON, RV>), dim3((unsigned)nblk), dim3(NT), 0, st, s, c, in,
                       out, partials, tiles_x, tiles_y, zchunk);
    return hipGetLastError();
}

template <int BC, int RV>
hipError_t launch_tb_mon(const Shape &s, const StepCoef &c, const double *in, double *out,
                         double *partials, int64_t *nparts, int zchunk, hipStream_t st)
{
    return partials ? launch_tb<BC, true, RV>(s, c, in, out, partials, nparts, zchunk, st)
                    : launch_tb<BC, false, RV>(s, c, in, out, partials, nparts, zchunk, st);
}

template <int BC>
hipError_t launch_tb_nit(const Shape &s, const StepCoef &c, const double *in, double *out,
                         double *partials, int64_t *nparts, int zchunk, hipStream_t st)
{
    switch (root_variant(c)) {
    case 1: return launch_tb_mon<BC, 1>(s, c, in, out, partials, nparts, zchunk, st);
    case 2: return launch_tb_mon<BC, 2>(s, c, in, out, partials, nparts, zchunk, st);
    case 3: return launch_tb_mon<BC, 3>(s, c, in, out, partials, nparts, zchunk, st);
    case 5: return launch_tb_mon<BC, 5>(s, c, in, out, partials, nparts, zchunk, st);
    case 6: return launch_tb_mon<BC, 6>(s, c, in, out, partials, nparts, zchunk, st);
    default: return launch_tb_mon<BC, 0>(s, c, in, out, partials, nparts, zchunk, st);
    }
}

}  // namespace

// zchunk > 0: one workgroup per (tile, chunk of zchunk planes); zchunk = 0:
// a persistent grid of the workgroups that fit at once, each marching an
// even share of the tile-planes (at least PERSIST_MIN of them).
hipError_t launch_step_tblock2(const Shape &s, const StepCoef &c, const double *in, double *out,
                               double *partials, int64_t *nparts, int zchunk, hipStream_t st)
{
    if (!tblock_supported(s) || zchunk < 0) return hipErrorInvalidValue;
    switch (s.bc) {
    case BC_HN: return launch_tb_nit<BC_HN>(s, c, in, out, partials, nparts, zchunk, st);
    case BC_HD: return launch_tb_nit<BC_HD>(s, c, in, out, partials, nparts, zchunk, st);
    case BC_P: return launch_tb_nit<BC_P>(s, c, in, out, partials, nparts, zchunk, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ace
