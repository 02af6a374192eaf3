// Internal declarations shared by the host runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ace {

enum { BC_HN = 0, BC_HD = 1, BC_P = 2 };

// Per-problem coefficients of one step (Sec. 2): kappa = eps^2 dt/dx^2,
// h = dt/2, omh = 1 - h, oph = 1 + h, h3 = 3 h (the cubic's derivative is
// 1 - h + 3 h theta^2), nit = Newton steps for |xi| <= 1, start2 = 1 when
// the root iteration starts from its second-order expansion in h, hs = the h
// of that expansion (h, or 0 when h > 1/2: the start is then |xi| itself).
struct StepCoef {
    double kappa;
    double h;
    double omh;
    double oph;
    double h3;
    double hs;
    int nit;
    int start2;
    int fex;    // 1: the fully explicit comparison scheme (no cubic solve)
    double dt;  // 2h, used by the explicit scheme
};

// Shape of one field: M[0] x M[1] x M[2] stored nodes in C order (unused
// leading axes are 1: a 2D field is 1 x M1 x M2, a 1D field 1 x 1 x M2).
struct Shape {
    int d;
    int bc;
    int64_t M0, M1, M2;
};

// ---- launchers (each defined next to its kernel) ---------------------------

// One step with one thread per node (neighbours through the cache).  If
// partials is not null, each block also writes (bulk, grad, max) of `in`
// to partials[3 * block ...] and *nparts receives the block count.
hipError_t launch_step_direct(const Shape &s, const StepCoef &c, const double *in,
                              double *out, double *partials, int64_t *nparts,
                              hipStream_t st);

int64_t direct_partials_needed(const Shape &s);  // blocks of launch_step_direct

// Monitor partials of a field without stepping.
hipError_t launch_monitor(const Shape &s, const double *in, double *partials,
                          int64_t *nparts, hipStream_t st);
int64_t monitor_partials_needed(const Shape &s);

// out[0] = dxd (trip[0] + cg trip[1]) (the energy), out[1] = trip[2].
hipError_t launch_monitor_finish(const double *trip, double dxd, double cg, double *out,
                                 hipStream_t st);

// Fixed-order reduction of nparts triples to one triple at out[0..2].
hipError_t launch_reduce(const double *partials, int64_t nparts, double *out,
                         hipStream_t st);

// Whole field in LDS: nsteps steps in one launch (total <= RESIDENT_MAX).
// When every > 0 the monitor triple of steps 0, every, ... <= nsteps is
// written to mon[3 j ...].  The result ends in `field` (in place).
constexpr int64_t RESIDENT_MAX = 8000;
hipError_t launch_resident(const Shape &s, const StepCoef &c, double *field,
                           int64_t nsteps, int64_t every, double *mon,
                           hipStream_t st);

// 2D/3D: tiles of the last two axes marching along axis 0 with the current
// plane in LDS and axis-0 neighbours in registers.  Same partials contract
// as launch_step_direct.
hipError_t launch_step_march(const Shape &s, const StepCoef &c, const double *in,
                             double *out, double *partials, int64_t *nparts,
                             hipStream_t st);
bool march_supported(const Shape &s);
int64_t march_partials_needed(const Shape &s);

// 3D: two steps per launch (temporal blocking); same partials contract (the
// monitors are those of the input field).  zchunk = planes per workgroup, or
// 0 for a persistent grid in which each workgroup marches an even share of
// all tile-planes.
hipError_t launch_step_tblock2(const Shape &s, const StepCoef &c, const double *in,
                               double *out, double *partials, int64_t *nparts, int zchunk,
                               hipStream_t st);
bool tblock_supported(const Shape &s);
int64_t tblock_partials_needed(const Shape &s, int zchunk);
constexpr int TBLOCK_MIN_ZCHUNK = 8;

// 3D: the configurable temporally blocked kernel (ace_tb3.h).  Variant v of
// TB3_TABLE advances `depth` steps per launch on regions of `rows` x 64
// nodes with `rpt` rows per thread (rows / rpt wavefronts per workgroup).
// Same partials contract (the monitors are those of the input field) and
// the same zchunk meaning as launch_step_tblock2.
struct Tb3Variant {
    int depth, rows, rpt;
};
constexpr int TB3_VARIANTS = 6;
constexpr Tb3Variant TB3_TABLE[TB3_VARIANTS] = {{2, 32, 4}, {3, 48, 3}, {3, 48, 4},
                                                {3, 32, 2}, {4, 32, 4}, {4, 32, 2}};
constexpr int TB3_DEFAULT_DEPTH3 = 1, TB3_DEFAULT_DEPTH4 = 5;  // variants ace_set_kernel picks
hipError_t launch_step_tb3(int v, const Shape &s, const StepCoef &c, const double *in, double *out,
                           double *partials, int64_t *nparts, int zchunk, hipStream_t st);
int64_t tb3_partials_needed(int v, const Shape &s, int zchunk);
bool tb3_supported(const Shape &s);  // d == 3 with planes of fewer than 2^31 nodes
int tb3_find(int depth, int rows, int rpt);  // variant index, or -1

// 2D: K steps per launch on LDS regions (1 <= K <= tblock2d_max_depth()).
// With level_stride > 0 every intermediate level k = 1..K is written to
// out + (k-1) * level_stride (the adjoint's segment recompute); otherwise only
// level K goes to out.  Same partials contract as the one-step kernels.
hipError_t launch_step_tblock2d(const Shape &s, const StepCoef &c, const double *in,
                                double *out, double *partials, int64_t *nparts, int K,
                                int64_t level_stride, hipStream_t st);
// 2D: the register-resident blocked kernel (ace_tb2.h).  Variant v of
// TB2_TABLE works on regions of `rows` x 64 nodes with `rpt` rows per thread
// and takes 1 <= K <= rows / 2 - 4 steps per launch; same contracts as
// launch_step_tblock2d.
struct Tb2Variant {
    int rows, rpt;
};
constexpr int TB2_VARIANTS = 4;
constexpr Tb2Variant TB2_TABLE[TB2_VARIANTS] = {{32, 4}, {32, 2}, {64, 4}, {16, 2}};
hipError_t launch_step_tb2(int v, const Shape &s, const StepCoef &c, const double *in, double *out,
                           double *partials, int64_t *nparts, int K, int64_t level_stride, hipStream_t st);
int64_t tb2_blocks(int v, const Shape &s, int K);
inline int tb2_max_depth(int v) { return TB2_TABLE[v].rows / 2 - 4; }
int tb2_find(int rows, int rpt);  // variant index, or -1
bool tb2_supported(const Shape &s);  // d == 2 with fewer than 2^31 nodes

// K transposed steps: states[i * stride] = phi^{m+i}, i = 0..K; lam_in =
// lambda^{m+K}; writes lambda^m and one partial of dL/dkappa per block.
hipError_t launch_adjoint_tblock2d(const Shape &s, const StepCoef &c, const double *lam_in,
                                   const double *states, int64_t stride, double *lam_out,
                                   double *gpart, int K, hipStream_t st);
bool tblock2d_supported(const Shape &s);
int tblock2d_max_depth();
int64_t tblock2d_blocks(const Shape &s, int K);

// Adjoint step (reverse sweep) for one step n: reads lam (lambda^{n+1}),
// phin (phi^n), phin1 (phi^{n+1}); writes lam_out (lambda^n) and per-block
// partial sums of <mu, Lambda phi^n> into gpart (count in *nparts).
hipError_t launch_adjoint_step(const Shape &s, const StepCoef &c, const double *lam,
                               const double *phin, const double *phin1,
                               double *lam_out, double *gpart, int64_t *nparts,
                               hipStream_t st);
int64_t adjoint_partials_needed(const Shape &s);
// out[0] = sum_i (1 + f_i)/2 over n values (fixed order, two passes through
// part, which holds phase_partials_needed() doubles).
int64_t phase_partials_needed();
hipError_t launch_phase_volume(const double *f, int64_t n, double *part, double *out,
                               hipStream_t st);
// Fixed-order sum of n doubles into out[0] (+= if accumulate).
hipError_t launch_sum(const double *x, int64_t n, double *out, int accumulate,
                      hipStream_t st);

}  // namespace ace
