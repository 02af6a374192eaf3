// 2D temporal blocking: K steps of the scheme (or K transposed steps) per
// launch on LDS-resident regions.
//
// A workgroup (512 threads: one wavefront per region row, eight thread rows,
// region row r handled by thread row r % 8) loads the 32 x 64 region around a
// (32 - 2K) x (64 - 2K) tile, with a ring of K nodes, into a padded LDS
// plane and advances it K times between two LDS buffers (one barrier per
// step).  After step k only rows [k, 32 - k) are still needed, so wavefronts
// skip the others.  The tile interior is exact after K steps and is written
// back (every level, when the caller wants all intermediate states).  Values
// outside the domain are loaded BC-mapped (clamped / zero / wrapped); for
// Neumann and Dirichlet an in-domain boundary node reads its outward
// neighbour from its own slot (mirror) or from the zero pad instead.  The
// arithmetic and the neighbour order are those of the one-step kernels, so
// results equal K one-step launches bit for bit.
//
// The transposed kernel walks K steps backwards on the same tiles:
//   mu = lambda / (1 + h (3 phi_{j+1}^2 - 1)),
//   lambda_j = (1 - h (3 phi_j^2 - 1)) mu + kappa Lambda mu,
//   g += < mu, Lambda phi_j > over the tile,
// reading the stored states phi_j, phi_{j+1} of each level into LDS.
#include <type_traits>

#include "ace_device.h"
#include "ace_tile2d.h"

namespace ace {

namespace {

using namespace tile2d;

constexpr int BTR = 8;           // thread rows
constexpr int BRT = BH / BTR;    // rows per thread
constexpr int BNT = BX * BTR;    // 512 threads

// RV: the root variant of cubic_root_n (start and Newton count fixed at
// compile time, identical rounding to the run-time path; 0: run time).
template <int BC, bool MON, bool LEVELS, int RV>
__global__ __launch_bounds__(BNT) void k_tblock2d(Shape s, StepCoef c, const double *__restrict__ in,
                                                  double *__restrict__ out,
                                                  double *__restrict__ partials, int K, int tiles_x,
                                                  int64_t level_stride)
{
    __shared__ double F[2 * BLP];
    __shared__ double red[3 * (BNT / 64)];
    const int tx = threadIdx.x & (BX - 1);
    const int tr = threadIdx.x / BX;
    const Geo g = make_geo<BC>(s, K, tiles_x, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x & (BX - 1));
    for (int i = threadIdx.x; i < 2 * BLP; i += BNT) F[i] = 0.0;
    __syncthreads();
    // level 0 into buffer 0
#pragma unroll
    for (int j = 0; j < BRT; ++j) {
        const int ry = tr + BTR * j;
        const int64_t o = goff<BC>(s, g.y0r + ry, g.xg);
        F[(ry + 1) * BLW + tx + 1] = (o < 0) ? 0.0 : in[o];
    }
    __syncthreads();
    MonAcc m;
    mon_zero(m);
    const bool xin = g.xg >= 0 && g.xg < s.M2 && tx >= K && tx < BX - K;
    if (MON) {
#pragma unroll
        for (int j = 0; j < BRT; ++j) {
            const int ry = tr + BTR * j;
            const int64_t yg = g.y0r + ry;
            if (!(xin && ry >= K && ry < BH - K && yg >= 0 && yg < s.M1)) continue;
            const int o = (ry + 1) * BLW + tx + 1;
            const double p = F[o];
            // next-node differences with the BC value past the end (the
            // loaded slot holds it), plus Dirichlet's first-node wall edge
            const double dy = F[o + BLW] - p, dx = F[o + 1] - p;
            double gr = fma(dy, dy, dx * dx);
            if (BC == BC_HD) {
                if (yg == 0) gr = fma(p, p, gr);
                if (g.xg == 0) gr = fma(p, p, gr);
            }
            m.bulk += bulk_term(p);
            m.grad += gr;
            m.mx = nan_max(m.mx, fabs(p));
        }
    }
    for (int k = 1; k <= K; ++k) {
        const double *src = F + ((k - 1) & 1) * BLP;
        double *dst = F + (k & 1) * BLP;
#pragma unroll
        for (int j = 0; j < BRT; ++j) {
            const int ry = tr + BTR * j;
            if (ry < k || ry >= BH - k) continue;  // wave-uniform
            int ym, yp;
            yoffs<BC>(s, g, ry, ym, yp);
            const int o = (ry + 1) * BLW + tx + 1;
            const double p = src[o];
            const double nsum = (src[o + ym] + src[o + yp]) + (src[o + g.xm] + src[o + g.xp]);
            const double v = update_n<2, RV>(p, nsum, c);
            dst[o] = v;
            if (LEVELS || k == K) {
                const int64_t yg = g.y0r + ry;
                if (xin && ry >= K && ry < BH - K && yg >= 0 && yg < s.M1)
                    out[(LEVELS ? (int64_t)(k - 1) * level_stride : 0) + yg * s.M2 + g.xg] = v;
            }
        }
        __syncthreads();
    }
    if (MON) block_reduce_store(m, red, partials + 3 * blockIdx.x);
}

// mu = lambda R'(xi): see ace_adjoint.hip (same refined reciprocal).
__device__ __forceinline__ double mu2(double lam, double p1, const StepCoef &c)
{
    const double dp = fma(c.h3, p1 * p1, c.omh);
    double r = __builtin_amdgcn_rcp(dp);
    r = fma(r, fma(-dp, r, 1.0), r);
    r = fma(r, fma(-dp, r, 1.0), r);
    return lam * r;
}

// K transposed steps.  lam_in = lambda^{m+K}; states[i * stride] = phi^{m+i},
// i = 0..K.  Writes lambda^m of the tile and the tile's sum of
// <mu, Lambda phi_j> over the K levels to gpart[block].
template <int BC>
__global__ __launch_bounds__(BNT) void k_adjoint_tb2d(Shape s, StepCoef c,
                                                      const double *__restrict__ lam_in,
                                                      const double *__restrict__ states,
                                                      int64_t stride, double *__restrict__ lam_out,
                                                      double *__restrict__ gpart, int K, int tiles_x)
{
    __shared__ double MU[BLP];
    __shared__ double P[2 * BLP];
    __shared__ double red[BNT / 64];
    const int tx = threadIdx.x & (BX - 1);
    const int tr = threadIdx.x / BX;
    const Geo g = make_geo<BC>(s, K, tiles_x, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x & (BX - 1));
    for (int i = threadIdx.x; i < BLP; i += BNT) {
        MU[i] = 0.0;
        P[i] = 0.0;
        P[BLP + i] = 0.0;
    }
    __syncthreads();
    int64_t goffs[BRT];
    double lam[BRT];
#pragma unroll
    for (int j = 0; j < BRT; ++j) {
        const int ry = tr + BTR * j;
        goffs[j] = goff<BC>(s, g.y0r + ry, g.xg);
        lam[j] = (goffs[j] < 0) ? 0.0 : lam_in[goffs[j]];
        P[BLP + (ry + 1) * BLW + tx + 1] = (goffs[j] < 0) ? 0.0 : states[(int64_t)K * stride + goffs[j]];
    }
    const bool xin = g.xg >= 0 && g.xg < s.M2 && tx >= K && tx < BX - K;
    // the stored state of the next level down is loaded into registers one
    // level ahead, so its latency overlaps the current level
    double nxt[BRT];
    auto fetch = [&](int i) {
#pragma unroll
        for (int j = 0; j < BRT; ++j) nxt[j] = (goffs[j] < 0) ? 0.0 : states[(int64_t)i * stride + goffs[j]];
    };
    fetch(K - 1);
    double gsum = 0.0;
    int cur1 = 1;  // buffer holding phi_{j+1}
    for (int i = K - 1; i >= 0; --i) {
        // phi_j into the other buffer
        double *p0 = P + (cur1 ^ 1) * BLP;
        const double *p1 = P + cur1 * BLP;
        const int lvl = K - 1 - i;  // reverse steps already taken
#pragma unroll
        for (int j = 0; j < BRT; ++j) {
            const int ry = tr + BTR * j;
            p0[(ry + 1) * BLW + tx + 1] = nxt[j];
        }
        if (i > 0) fetch(i - 1);
        // mu of the region rows still exact
#pragma unroll
        for (int j = 0; j < BRT; ++j) {
            const int ry = tr + BTR * j;
            if (ry < lvl || ry >= BH - lvl) continue;
            const int o = (ry + 1) * BLW + tx + 1;
            MU[o] = mu2(lam[j], p1[o], c);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < BRT; ++j) {
            const int ry = tr + BTR * j;
            if (ry < lvl + 1 || ry >= BH - lvl - 1) continue;
            int ym, yp;
            yoffs<BC>(s, g, ry, ym, yp);
            const int o = (ry + 1) * BLW + tx + 1;
            const double mu = MU[o];
            const double p = p0[o];
            const double msum = (MU[o + ym] + MU[o + yp]) + (MU[o + g.xm] + MU[o + g.xp]);
            const double lap_mu = fma(-4.0, mu, msum);
            const double jd = fma(-c.h3, p * p, 1.0 + c.h);
            lam[j] = fma(c.kappa, lap_mu, jd * mu);
            const int64_t yg = g.y0r + ry;
            if (xin && ry >= K && ry < BH - K && yg >= 0 && yg < s.M1) {
                const double psum = (p0[o + ym] + p0[o + yp]) + (p0[o + g.xm] + p0[o + g.xp]);
                gsum += mu * fma(-4.0, p, psum);
            }
        }
        __syncthreads();
        cur1 ^= 1;
    }
#pragma unroll
    for (int j = 0; j < BRT; ++j) {
        const int ry = tr + BTR * j;
        const int64_t yg = g.y0r + ry;
        if (xin && ry >= K && ry < BH - K && yg >= 0 && yg < s.M1) lam_out[yg * s.M2 + g.xg] = lam[j];
    }
    gsum = wave_sum(gsum);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = gsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int w = 1; w < BNT / 64; ++w) t += red[w];
        gpart[blockIdx.x] = t;
    }
}

void tiles2d(const Shape &s, int K, int &tiles_x, int &ntiles)
{
    const int oy = BH - 2 * K, ox = BX - 2 * K;
    tiles_x = (int)((s.M2 + ox - 1) / ox);
    ntiles = tiles_x * (int)((s.M1 + oy - 1) / oy);
}

}  // namespace

int tblock2d_max_depth() { return BH / 2 - 4; }  // keeps a 8 x 56 tile at least

bool tblock2d_supported(const Shape &s) { return s.d == 2 && s.M1 >= 1 && s.M2 >= 1; }

int64_t tblock2d_blocks(const Shape &s, int K)
{
    int tx, n;
    tiles2d(s, K, tx, n);
    return n;
}

namespace {

template <int BC, int RV>
hipError_t launch_t2(const Shape &s, const StepCoef &c, const double *in, double *out, double *partials,
                     int K, int tiles_x, int ntiles, int64_t level_stride, bool levels, hipStream_t st)
{
    if (partials)
        hipLaunchKernelGGL((k_tblock2d<BC, true, false, RV>), dim3(ntiles), dim3(BNT), 0, st, s, c, in,
                           out, partials, K, tiles_x, level_stride);
    else if (levels)
        hipLaunchKernelGGL((k_tblock2d<BC, false, true, RV>), dim3(ntiles), dim3(BNT), 0, st, s, c, in,
                           out, partials, K, tiles_x, level_stride);
    else
        hipLaunchKernelGGL((k_tblock2d<BC, false, false, RV>), dim3(ntiles), dim3(BNT), 0, st, s, c, in,
                           out, partials, K, tiles_x, level_stride);
    return hipGetLastError();
}

template <int BC>
hipError_t launch_t2_nit(const Shape &s, const StepCoef &c, const double *in, double *out,
                         double *partials, int K, int tiles_x, int ntiles, int64_t level_stride,
                         bool levels, hipStream_t st)
{
    const int rv = root_variant(c);
    auto go = [&](auto tag) {
        return launch_t2<BC, decltype(tag)::value>(s, c, in, out, partials, K, tiles_x, ntiles, level_stride,
                                                   levels, st);
    };
    switch (rv) {
    case 1: return go(std::integral_constant<int, 1>());
    case 2: return go(std::integral_constant<int, 2>());
    case 3: return go(std::integral_constant<int, 3>());
    case 5: return go(std::integral_constant<int, 5>());
    case 6: return go(std::integral_constant<int, 6>());
    default: return go(std::integral_constant<int, 0>());
    }
}

}  // namespace

hipError_t launch_step_tblock2d(const Shape &s, const StepCoef &c, const double *in, double *out,
                                double *partials, int64_t *nparts, int K, int64_t level_stride,
                                hipStream_t st)
{
    if (!tblock2d_supported(s) || K < 1 || K > tblock2d_max_depth()) return hipErrorInvalidValue;
    int tiles_x, ntiles;
    tiles2d(s, K, tiles_x, ntiles);
    if (nparts) *nparts = ntiles;
    const bool levels = level_stride > 0;
    switch (s.bc) {
    case BC_HN:
        return launch_t2_nit<BC_HN>(s, c, in, out, partials, K, tiles_x, ntiles, level_stride, levels, st);
    case BC_HD:
        return launch_t2_nit<BC_HD>(s, c, in, out, partials, K, tiles_x, ntiles, level_stride, levels, st);
    case BC_P:
        return launch_t2_nit<BC_P>(s, c, in, out, partials, K, tiles_x, ntiles, level_stride, levels, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_tblock2d(const Shape &s, const StepCoef &c, const double *lam_in,
                                   const double *states, int64_t stride, double *lam_out,
                                   double *gpart, int K, hipStream_t st)
{
    if (!tblock2d_supported(s) || K < 1 || K > tblock2d_max_depth()) return hipErrorInvalidValue;
    int tiles_x, ntiles;
    tiles2d(s, K, tiles_x, ntiles);
#define ACE_A2(BB)                                                                          \
    if (s.bc == BB) {                                                                       \
        hipLaunchKernelGGL((k_adjoint_tb2d<BB>), dim3(ntiles), dim3(BNT), 0, st, s, c, lam_in, \
                           states, stride, lam_out, gpart, K, tiles_x);                     \
        return hipGetLastError();                                                           \
    }
    ACE_A2(BC_HN) ACE_A2(BC_HD) ACE_A2(BC_P)
#undef ACE_A2
    return hipErrorInvalidValue;
}

}  // namespace ace
