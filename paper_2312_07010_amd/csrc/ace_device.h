// Device-side building blocks of the RLB-MIE-FD step for gfx950 (wave64).
//
// The step (Sec. 2, pointwise form IE-FD) at a node with value p is
//   xi    = p + kappa * sum_k (p_{+k} + p_{-k} - 2 p) - h (p^3 - p),
//   p_new = the unique real root theta of theta + h (theta^3 - theta) = xi
// (Sec. 3.2, Remark 1: unique for 0 < dt < 2), with h = dt/2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ace_internal.h"

namespace ace {

// Reciprocal of a positive double near [0.5, 4]: hardware estimate plus one
// Newton-Raphson correction.  Only used for Newton steps on the cubic, whose
// own iteration absorbs the remaining error.
__device__ __forceinline__ double approx_rcp(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    const double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    return r;
}

// Unique real root of theta + h (theta^3 - theta) = xi for 0 < h < 1.
// The root map is odd, so the iteration runs on a = |xi| and the sign is
// restored.  For a <= 1 (always the case under Theorem 2's conditions) it
// starts from the expansion of the root in h, to first order,
// theta_0 = a - h f(a) = a + h a (1 - a^2), or (c.start2) to second order,
// theta_0 = a - h f(a) (1 - h f'(a)) with f' = 3 a^2 - 1, and takes `nit`
// Newton steps on the cubic; the host picks the start and nit by running
// this same iteration in extended precision over a <= 1.  When h > 1/2 the
// expansion is poor and the start is a itself: the expansion's h is then
// c.hs = 0, which gives a exactly (a + 0 * (finite) = a), so no lane selects.
// 0 and 1 are exact fixed points of both starts and of the step
// (f(0) = f(1) = 0), so 0 and +-1 are returned exactly.  For a > 1 (only
// when the conditions fail) the iteration starts from a instead, takes the
// same `nit` steps and continues until the correction stops mattering (at
// most 200 more steps).
template <bool S2>
__device__ __forceinline__ double root_start_t(double a, const StepCoef &c)
{
    if (S2) {
        const double a2 = a * a;
        const double f = fma(a2, a, -a);        // f(a)
        const double t = fma(-c.h3, a2, c.oph);  // 1 - h f'(a)
        return fma(-(c.hs * f), t, a);
    }
    return fma(c.hs * a, fma(-a, a, 1.0), a);
}

__device__ __forceinline__ double root_start(double a, const StepCoef &c)
{
    return c.start2 ? root_start_t<true>(a, c) : root_start_t<false>(a, c);
}

// Root variants fixed at compile time: RV = NIT + 4 * START2, with NIT = 1..3
// Newton steps and START2 the second-order start; RV = 0 takes both from the
// coefficients at run time.  root_variant() gives a launcher the RV of a
// coefficient set (0 for combinations without an instantiation: the explicit
// scheme, and nit > 3).
__host__ __device__ inline int root_variant(const StepCoef &c)
{
    if (c.fex || c.nit < 1 || c.nit > 3 || (c.start2 && c.nit == 3)) return 0;
    return c.nit + 4 * c.start2;
}

// A copy of c with omh and oph held in vector registers.  A VOP3
// instruction reads at most one scalar register, so fma(h3, x^2, omh) of the
// Newton step and fma(-h3, a^2, oph) of the second-order start, with both
// coefficients in scalar registers, cost a move at every node; a kernel that
// passes this copy to the root pays those moves once.  (The empty asm only
// makes the values look per-lane to the compiler; it emits no instruction.)
__device__ __forceinline__ StepCoef coef_vgpr(const StepCoef &c)
{
    StepCoef v = c;
    asm volatile("" : "+v"(v.omh), "+v"(v.oph));
    return v;
}

// One Newton step on the cubic from x, with the reciprocal of the
// derivative from its hardware estimate and one correction.
__device__ __forceinline__ double newton_step(double x, double a, const StepCoef &c)
{
    const double x2 = x * x;
    const double p = fma(c.h, fma(x, x2, -x), x - a);
    const double dp = fma(c.h3, x2, c.omh);
    return fma(-p, approx_rcp(dp), x);
}

// Newton steps with a true division from x until the correction stops
// mattering (below 2^-54 x; at most 200 steps): the root for a > 1.
__device__ __forceinline__ double newton_converge(double x, double a, const StepCoef &c)
{
    for (int k = 0; k < 200; ++k) {
        const double x2 = x * x;
        const double p = fma(c.h, fma(x, x2, -x), x - a);
        const double dp = fma(c.h3, x2, c.omh);
        const double step = p / dp;
        x -= step;
        if (!(fabs(step) > 0x1p-54 * x)) break;
    }
    return x;
}

// (With the step count known only at run time, a lane with a > 1 selects
// the start a and goes on after the common steps, in less code than the
// restart of cubic_root_n for kernels that inline many roots; the
// arithmetic is the same.)
__device__ __forceinline__ double cubic_root(double xi, const StepCoef &c)
{
    const double a = fabs(xi);
    double x = a > 1.0 ? a : root_start(a, c);
    for (int k = 0; k < c.nit; ++k) x = newton_step(x, a, c);
    if (a > 1.0) x = newton_converge(x, a, c);
    return copysign(x, xi);
}

// The root's two paths for a = |xi| with the start and the Newton count
// fixed at compile time (RV > 0, see root_variant): root_common is the start
// and NIT steps, the root for a <= 1; root_restart the root for a > 1 (from
// a, the same NIT steps, then newton_converge).  The iteration and hence
// every rounding is identical to cubic_root's with the matching
// coefficients, so the loop unrolls and its constants stay in registers.
template <int RV>
__device__ __forceinline__ double root_common(double a, const StepCoef &c)
{
    constexpr int NIT = RV > 0 ? (RV & 3) : 1;
    double x = root_start_t<(RV >= 4)>(a, c);
#pragma unroll
    for (int k = 0; k < NIT; ++k) x = newton_step(x, a, c);
    return x;
}

template <int RV>
__device__ __forceinline__ double root_restart(double a, const StepCoef &c)
{
    constexpr int NIT = RV > 0 ? (RV & 3) : 1;
    double x = a;
#pragma unroll
    for (int k = 0; k < NIT; ++k) x = newton_step(x, a, c);
    return newton_converge(x, a, c);
}

template <int RV>
__device__ __forceinline__ double cubic_root_n(double xi, const StepCoef &c)
{
    if (RV <= 0) return cubic_root(xi, c);
    const double a = fabs(xi);
    double x = root_common<RV>(a, c);
    if (a > 1.0) x = root_restart<RV>(a, c);  // this lane's first pass is discarded
    return copysign(x, xi);
}

// The roots of N values with one test for the a > 1 case (on the largest
// |xi|; a NaN never needs it), so the common paths of the N values form one
// block that the compiler can interleave.  Same results as cubic_root_n.
template <int RV, int N>
__device__ __forceinline__ void cubic_roots_n(const double (&xi)[N], double (&th)[N], const StepCoef &c)
{
    double amax = fabs(xi[0]);
#pragma unroll
    for (int r = 0; r < N; ++r) {
        th[r] = root_common<RV>(fabs(xi[r]), c);
        if (r > 0) amax = fmax(amax, fabs(xi[r]));
    }
    if (amax > 1.0) {
#pragma unroll
        for (int r = 0; r < N; ++r)
            if (fabs(xi[r]) > 1.0) th[r] = root_restart<RV>(fabs(xi[r]), c);
    }
#pragma unroll
    for (int r = 0; r < N; ++r) th[r] = copysign(th[r], xi[r]);
}

// Explicit part xi from the node value p and the sum over axes of its two
// neighbours' sum (nsum = sum_k (p_{+k} + p_{-k})), for d = D.
template <int D>
__device__ __forceinline__ double explicit_part(double p, double nsum, const StepCoef &c)
{
    const double lap = fma(-2.0 * D, p, nsum);
    const double t = fma(c.kappa, lap, p);
    const double f = fma(p, p * p, -p);
    return fma(-c.h, f, t);
}

// The fully explicit comparison scheme of Sec. 3.3, Remark 2 (FEX-FD):
// phi + kappa sum_k (phi_{+k} + phi_{-k} - 2 phi) - dt f(phi).
template <int D>
__device__ __forceinline__ double explicit_fex(double p, double nsum, const StepCoef &c)
{
    const double lap = fma(-2.0 * D, p, nsum);
    const double t = fma(c.kappa, lap, p);
    const double f = fma(p, p * p, -p);
    return fma(-c.dt, f, t);
}

template <int D>
__device__ __forceinline__ double update(double p, double nsum, const StepCoef &c)
{
    if (c.fex) return explicit_fex<D>(p, nsum, c);
    return cubic_root(explicit_part<D>(p, nsum, c), c);
}

// (RV > 0 implies the implicit scheme: root_variant gives 0 for the explicit
// one, so only RV = 0 tests c.fex.)
template <int D, int RV>
__device__ __forceinline__ double update_n(double p, double nsum, const StepCoef &c)
{
    if (RV <= 0 && c.fex) return explicit_fex<D>(p, nsum, c);
    return cubic_root_n<RV>(explicit_part<D>(p, nsum, c), c);
}

// Value used for an out-of-range neighbour (rows of the paper's D matrices):
// Neumann mirrors the node itself, Dirichlet reads the zero wall, periodic
// reads the wrapped node `wrap`.
template <int BC>
__device__ __forceinline__ double outside(double self, double wrap)
{
    if (BC == BC_HN) return self;
    if (BC == BC_HD) return 0.0;
    return wrap;
}

// NaN-propagating maximum (fmax drops NaN).
// Workgroups are dealt to the 8 XCDs round-robin: block b runs on XCD b % 8.
// This renumbering gives each XCD one contiguous range of logical tiles, so
// neighbouring tiles, which read each other's edge rows, share that XCD's L2.
// It is a bijection on [0, nblk) for every nblk: with nblk = 8q + r, XCDs
// 0..r-1 take q+1 tiles and the others q.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nblk)
{
    const int64_t q = nblk >> 3, r = nblk & 7, x = b & 7, k = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

__device__ __forceinline__ double nan_max(double a, double b)
{
    if (a != a) return a;
    if (b != b) return b;
    return a > b ? a : b;
}

// Monitor terms of one node with value p: bulk (p^2 - 1)^2 / 4; the squared
// difference along each axis to the next node (the BC's value past the last
// node, so HN adds 0, HD adds p^2 for the wall edge, P adds the wrap edge);
// HD also adds p^2 for the wall edge before the first node.
struct MonAcc {
    double bulk, grad, mx;
};

__device__ __forceinline__ void mon_zero(MonAcc &m)
{
    m.bulk = 0.0;
    m.grad = 0.0;
    m.mx = 0.0;
}

__device__ __forceinline__ double bulk_term(double p)
{
    const double q = fma(p, p, -1.0);
    return 0.25 * (q * q);
}

// Wave64 butterfly sums: every lane ends with the same, order-fixed value.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = nan_max(v, __shfl_xor(v, o, 64));
    return v;
}

// Deterministic block reduction of (bulk, grad, max); thread 0 writes the
// triple to out[0..2].  `lds` holds 3 * (blockDim / 64) doubles.
__device__ __forceinline__ void block_reduce_store(MonAcc m, double *lds, double *out)
{
    const int lane = threadIdx.x & 63;
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int wave = tid >> 6;
    const int nw = (nthreads + 63) >> 6;
    (void)lane;
    const double b = wave_sum(m.bulk);
    const double g = wave_sum(m.grad);
    const double x = wave_max(m.mx);
    if ((tid & 63) == 0) {
        lds[3 * wave + 0] = b;
        lds[3 * wave + 1] = g;
        lds[3 * wave + 2] = x;
    }
    __syncthreads();
    if (tid == 0) {
        double sb = 0.0, sg = 0.0, sx = 0.0;
        for (int w = 0; w < nw; ++w) {
            sb += lds[3 * w + 0];
            sg += lds[3 * w + 1];
            sx = nan_max(sx, lds[3 * w + 2]);
        }
        out[0] = sb;
        out[1] = sg;
        out[2] = sx;
    }
}

}  // namespace ace
