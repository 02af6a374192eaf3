/*
 * ace.h - C ABI of the MI355X (gfx950) FP64 solver for the RLB-MIE-FD scheme
 * of Chen, Liu, Chai and Shi (arXiv 2312.07010) for the d = 1, 2, 3
 * Allen-Cahn equation  phi_t = eps^2 lap(phi) - (phi^3 - phi).
 *
 * All functions are extern "C", take plain host or device pointers and sizes,
 * and return an int status: ACE_OK (0), a negative error (nothing changed
 * unless stated), or a positive warning (the call completed).  Handles are not
 * thread-safe; separate handles are independent.  Device pointers are HIP
 * device memory on the device that was current when the handle was created.
 *
 * Notation: N = cells per axis, dx = (R - L)/N (equal on every axis),
 * kappa = eps^2 dt / dx^2 (the paper's omega_1/s), h = dt/2,
 * f(phi) = phi^3 - phi.  Fields are stored in C order (last index fastest),
 * the paper's vector ordering (Sec. 2, vector form of the scheme).
 */
#ifndef ACE_H
#define ACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define ACE_OK 0
#define ACE_E_ARG (-1)       /* bad argument (null, d, L >= R, eps <= 0, ...) */
#define ACE_E_SIZE (-2)      /* too few cells for the boundary condition      */
#define ACE_E_ANISO (-3)     /* dx differs between axes                        */
#define ACE_E_DT (-4)        /* dt <= 0 or dt >= 2: the cubic has no unique root */
#define ACE_E_HIP (-5)       /* a HIP runtime call failed                      */
#define ACE_E_NOMEM (-6)     /* device or host allocation failed               */
#define ACE_E_NONFINITE (-7) /* NaN or Inf in a field                          */
#define ACE_E_STATE (-8)     /* call not valid in the handle's current state   */
#define ACE_W_CONDITIONS 1   /* dt > 1 - 2 d kappa or kappa >= 1/(2d): Theorem 2's
                                step condition fails (the run is still allowed) */
#define ACE_W_PHI0_GT1 2     /* |phi0| > 1 somewhere: Theorem 2's hypothesis fails */
#define ACE_W_MAXPRINCIPLE 3 /* a monitored max-norm exceeded 1 + 4 u while the
                                conditions hold                                 */
#define ACE_W_ENERGY_UP 4    /* a monitored energy rose by more than 1e-14 E
                                while the conditions hold                       */

/* ---- boundary conditions (Sec. 1; D matrices of Sec. 2) ----------------- */
#define ACE_BC_HN 0 /* homogeneous Neumann: N+2 nodes at L + (i - 1/2) dx     */
#define ACE_BC_HD 1 /* homogeneous Dirichlet: N-1 nodes at L + i dx, i=1..N-1 */
#define ACE_BC_P 2  /* periodic: N nodes at L + i dx, i = 0..N-1               */

/* ---- where a pointer lives --------------------------------------------- */
#define ACE_HOST 0
#define ACE_DEVICE 1

/* ---- kernel selection (ace_set_kernel) --------------------------------- */
#define ACE_KERNEL_AUTO 0    /* the autotuned / default choice                */
#define ACE_KERNEL_DIRECT 1  /* one thread per node, neighbours from cache    */
#define ACE_KERNEL_MARCH 2   /* 3D: tiles marching along axis 0, LDS planes    */
#define ACE_KERNEL_RESIDENT 3 /* whole field in LDS, many steps per launch    */
#define ACE_KERNEL_TBLOCK 4  /* temporal blocking: 3D 2..4 steps per launch,
                                2D 1..12 steps per launch                     */

/* ---- schemes (ace_set_scheme) ------------------------------------------ */
#define ACE_SCHEME_RLB_MIE 0 /* the paper's scheme (default)                   */
#define ACE_SCHEME_FEX 1     /* fully explicit comparison scheme (Remark 2)     */

typedef struct ace_solver ace_solver;

/* Derived parameters of a handle (Sec. 2 and Theorem 2 of Sec. 3.2). */
typedef struct {
    int d;              /* dimension 1..3                                    */
    int bc;             /* ACE_BC_*                                          */
    int64_t N[3];       /* cells per axis (unused axes 1)                    */
    int64_t M[3];       /* stored nodes per axis (unused axes 1)             */
    int64_t total;      /* product of M                                      */
    double dx, dt, eps; /* spacing, time step, interface width              */
    double kappa;       /* eps^2 dt / dx^2                                   */
    double h;           /* dt / 2                                            */
    double dt_bound;    /* largest dt with dt <= 1 - 2 d eps^2 dt/dx^2:
                           dx^2 / (dx^2 + 2 d eps^2)                          */
    double omega1;      /* the paper's weight choice 1/3, 1/5, 1/6 (Sec. 4)  */
    double s;           /* relaxation parameter omega1 / kappa              */
    int conditions_ok;  /* 1 if dt <= (1 - 2 d kappa)(1 + 1e-12) and
                           0 < kappa < 1/(2d)                                 */
    int newton_iters;   /* Newton steps of the pointwise cubic solve         */
    int scheme;         /* ACE_SCHEME_*                                      */
} ace_params_t;

/* ---- handle lifecycle --------------------------------------------------- */

/* Creates a solver for the problem of Sec. 1 on Omega = prod (L[j], R[j])
 * with N[j] cells per axis, interface width eps > 0, time step 0 < dt < 2 and
 * one boundary condition bc for the whole boundary.  Allocates two device
 * field buffers (C order, ace_shape nodes) and monitor scratch on the current
 * device and stream 0.  *out receives the handle (free with ace_destroy).
 * Errors: ACE_E_ARG (null pointers, d not 1..3, L >= R, eps <= 0, non-finite
 * input, bc unknown), ACE_E_SIZE (HN N < 1, HD N < 2, P N < 3),
 * ACE_E_ANISO (dx differs across axes by more than 1e-12 relative),
 * ACE_E_DT, ACE_E_HIP / ACE_E_NOMEM.  Warning: ACE_W_CONDITIONS. */
int ace_create(int d, const int64_t *N, const double *L, const double *R,
               double eps, double dt, int bc, ace_solver **out);

/* Frees the handle and the device memory it owns (not bound buffers). */
int ace_destroy(ace_solver *s);

/* Stored nodes per axis M[0..2] (unused axes 1) and their product. */
int ace_shape(const ace_solver *s, int64_t M[3], int64_t *total);

/* Coordinates of the stored nodes along axis (Sec. 2, grid function space):
 * x must hold M[axis] doubles (host). */
int ace_node_coords(const ace_solver *s, int axis, double *x);

/* Copies the derived parameters to *p (host). */
int ace_params(const ace_solver *s, ace_params_t *p);

/* Runs all later device work of the handle on this HIP stream (hipStream_t,
 * may be NULL for the default stream).  Switching to another stream first
 * waits for the old one and drops the graphs captured for it, so no replay
 * still in flight there loses its graph. */
int ace_set_stream(ace_solver *s, void *hip_stream);

/* Uses caller-owned device buffers a, b (each ace_shape total doubles) as
 * the two field buffers from now on; the handle never frees them.  The
 * current field is lost: call ace_set_phi0 next.  Both NULL reverts to the
 * handle's own buffers. */
int ace_bind_fields(ace_solver *s, double *a, double *b);

/* Changes the interface width eps > 0 (hence kappa = eps^2 dt / dx^2 and the
 * condition flag) keeping the field and the step counter; used when eps^2 is
 * trained.  Errors: ACE_E_ARG.  Warning: ACE_W_CONDITIONS. */
int ace_set_eps(ace_solver *s, double eps);

/* Runs of ace_step longer than twice `launches` launches are replayed from a
 * HIP graph holding `launches` step launches (rounded up to even), captured
 * on first use for the handle's current buffers and kernel; 0 disables graph
 * replay (every launch is issued directly).  Default 32.  Results are
 * identical either way. */
int ace_set_graph_launches(ace_solver *s, int64_t launches);

/* Selects the time step.  ACE_SCHEME_RLB_MIE (default) is the paper's scheme.
 * ACE_SCHEME_FEX is the fully explicit comparison scheme of Sec. 3.3,
 * Remark 2, phi^{n+1} = phi + kappa sum_k (phi_{+k} + phi_{-k} - 2 phi)
 * - dt f(phi), whose condition is dt <= (1 - 2 d kappa)/2; every kernel
 * choice supports both.  The reverse sweep supports only ACE_SCHEME_RLB_MIE.
 * Warning: ACE_W_CONDITIONS. */
int ace_set_scheme(ace_solver *s, int scheme);

/* Kernel choice for ace_step (ACE_KERNEL_*) and its temporal depth (steps
 * per launch; 0 = default).  ACE_KERNEL_TBLOCK accepts 0, 2, 3 or 4 in 3D
 * (2: the two-step kernel; 3, 4: the configurable kernel on its default
 * region for that depth, see ace_set_region3d) and 0..12 in 2D.  A choice
 * that does not apply to the handle's dimension or size falls back to
 * ACE_KERNEL_DIRECT.  Every choice computes the same result bit for bit.
 * Error: ACE_E_ARG for an unknown kernel or depth. */
int ace_set_kernel(ace_solver *s, int kernel, int depth);

/* Temporal depth and region shape of the 3D blocked kernel (launch
 * configuration only; results are unchanged bit for bit).  depth 2 with
 * rows = rows_per_thread = 0 selects the two-step kernel (regions of
 * 32 x 64 nodes, LDS planes double-buffered).  Otherwise (depth, rows,
 * rows_per_thread) names one instantiated variant of the configurable
 * kernel, which advances `depth` steps per launch on regions of rows x 64
 * nodes held in registers, rows_per_thread consecutive rows per thread
 * (rows / rows_per_thread wavefronts per workgroup), with a ring of depth
 * nodes recomputed: (2, 32, 4), (3, 48, 3), (3, 48, 4), (3, 32, 2),
 * (4, 32, 4), (4, 32, 2).  ace_autotune chooses among all of them.  Runs
 * shorter than the depth, and planes (M1 * M2) of 2^28 nodes or more, take
 * the two-step or one-step kernel.  Error:
 * ACE_E_ARG when d != 3 or the triple is not instantiated. */
int ace_set_region3d(ace_solver *s, int depth, int rows, int rows_per_thread);
int ace_get_region3d(const ace_solver *s, int *depth, int *rows, int *rows_per_thread);

/* Region shape of the 2D blocked kernel (launch configuration only; results
 * are unchanged bit for bit).  rows = rows_per_thread = 0 selects the kernel
 * that keeps each level's 32 x 64 region in LDS.  Otherwise (rows,
 * rows_per_thread) names one instantiated variant of the register-resident
 * kernel, which holds rows x 64 regions in registers, rows_per_thread
 * consecutive rows per thread, neighbours along a row moved between lanes
 * and across wavefronts through LDS edge rows: (32, 4), (32, 2), (64, 4),
 * (16, 2).  Its depth (ace_set_kernel) is capped at rows / 2 - 4.
 * ace_autotune chooses among all of them.  Error: ACE_E_ARG when d != 2 or
 * the pair is not instantiated. */
int ace_set_region2d(ace_solver *s, int rows, int rows_per_thread);
int ace_get_region2d(const ace_solver *s, int *rows, int *rows_per_thread);

/* Planes of axis 0 per workgroup of the 3D temporally blocked kernel
 * (launch shape only; results are unchanged).  0 selects a persistent grid:
 * as many workgroups as fit on the device at once, each marching an even
 * share of all (tile, plane) pairs.  ace_autotune sets it; this fixes it,
 * e.g. to take hardware counters of one launch shape.  planes = 0 or in
 * [8, 4096]; ACE_E_ARG otherwise or when d != 3. */
int ace_set_plane_chunk(ace_solver *s, int planes);

/* The plane chunk the 3D temporally blocked kernel will use. */
int ace_get_plane_chunk(const ace_solver *s, int *planes);

/* The kernel ace_step will actually use (after ACE_KERNEL_AUTO, the autotuned
 * choice and fallbacks are resolved) and its steps per launch. */
int ace_get_kernel(const ace_solver *s, int *kernel, int *steps_per_launch);

/* ---- the time step (Sec. 2, scheme IE-FD; Sec. 3.2, Remark 1) ------------ */

/* Sets phi^0 from total doubles in C order at phi0 (ACE_HOST: synchronous
 * copy; ACE_DEVICE: stream-ordered copy) and resets the step counter.
 * Errors: ACE_E_NONFINITE (host copies are checked).  Warning:
 * ACE_W_PHI0_GT1 (host copies). */
int ace_set_phi0(ace_solver *s, const double *phi0, int where);

/* Advances the field by nsteps >= 0 steps of
 *   phi^{n+1} + h f(phi^{n+1}) = phi^n + kappa sum_k (phi_{+k} + phi_{-k}
 *                                 - 2 phi) - h f(phi^n),
 * solving the monotone cubic for its unique real root per node.  Out-of-range
 * neighbours: HN mirror (the node itself), HD zero, P wrap.  Asynchronous on
 * the handle's stream. */
int ace_step(ace_solver *s, int64_t nsteps);

/* Advances by nsteps and records the discrete energy (Theorem 3) and the
 * max-norm at steps 0, every, 2 every, ... <= nsteps into host arrays E and
 * maxn of length nsteps/every + 1 (every >= 1).  The monitors of the field
 * a step reads are fused into that step.  Synchronous.  Errors:
 * ACE_E_NONFINITE.  Warnings (conditions_ok only): ACE_W_MAXPRINCIPLE,
 * ACE_W_ENERGY_UP; when both occur the return value is ACE_W_MAXPRINCIPLE
 * and ace_get_warnings reports both. */
int ace_run_monitored(ace_solver *s, int64_t nsteps, int64_t every,
                      double *E, double *maxn);

/* Bit of warning w in a warning mask. */
#define ACE_WARN_BIT(w) (1 << (w))

/* Every warning the last ace_run_monitored of the handle saw, as a mask of
 * ACE_WARN_BIT(ACE_W_MAXPRINCIPLE) and ACE_WARN_BIT(ACE_W_ENERGY_UP) (0 if
 * none or if no monitored run happened yet).  Host memory. */
int ace_get_warnings(const ace_solver *s, int *mask);

/* The check ace_run_monitored applies to its monitor series, on host
 * arrays E and maxn of n >= 1 values (steps 0, every, 2 every, ...):
 * under the step conditions (conditions_ok != 0) a max-norm above
 * 1 + 4 u (u = 2^-53) violates Theorem 2 (Sec. 3.2) and an energy rise
 * E[j] > E[j-1] + 1e-14 |E[j-1]| violates Theorem 3 (Sec. 3.3).  Writes
 * the mask of every warning seen to *mask (may be NULL) and returns
 * ACE_E_NONFINITE if any value is NaN or infinite, else ACE_W_MAXPRINCIPLE,
 * else ACE_W_ENERGY_UP, else ACE_OK.  Host-only: no device is touched. */
int ace_monitor_status(int64_t n, const double *E, const double *maxn,
                       int conditions_ok, int *mask);

/* Discrete energy of the current field (Sec. 3.3, Theorem 3):
 *   E = dx^d [ sum_i (phi_i^2 - 1)^2 / 4 - kappa/(2 dt) Phi^T Lambda Phi ],
 * with -Phi^T Lambda Phi the sum of squared differences over lattice edges
 * (HD includes the edges to the zero walls, P the wrap edges).  Deterministic
 * fixed-order reduction.  Synchronous; *E is host memory. */
int ace_energy(ace_solver *s, double *E);

/* max_i |phi_i| of the current field (Sec. 3.2, Theorem 2).  NaN if any node
 * is NaN.  Synchronous; *m is host memory. */
int ace_maxnorm(ace_solver *s, double *m);

/* Volume of the phase phi > 0, measured smoothly as dx^d sum_i (1 + phi_i)/2
 * (an odd interface profile makes this the volume inside the zero level
 * set); from it the equivalent radius of the shrinking circle / sphere of
 * the mean-curvature examples (Sec. 4.2.2).  Deterministic reduction.
 * Synchronous; *V is host memory. */
int ace_phase_volume(ace_solver *s, double *V);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * energy of ace_energy and the max-norm of ace_maxnorm, written to device
 * memory out[0] (energy) and out[1] (max-norm) by kernels on the handle's
 * stream, with no host synchronisation and no allocation.  phi is a device
 * field of the handle's shape (total doubles, C order) or NULL for the
 * handle's current field.  The per-block partial sums go to a static
 * scratch array of 1.5 MiB that each device holds for the life of the
 * process, shared by every handle on that device: calls that overlap on one
 * device (on different streams, or from different threads) race, and must
 * be ordered by the caller.  The values equal those of ace_energy and
 * ace_maxnorm bit for bit.  Errors: ACE_E_ARG (NULL handle or out),
 * ACE_E_SIZE (the field needs more than 65536 partial sums, about
 * 2^31 nodes in 3D, 2^26 in 2D and 2^24 in 1D), ACE_E_STATE (the scratch
 * address could not be looked up when the handle was created), ACE_E_HIP. */
int ace_monitor_noalloc(ace_solver *s, const double *phi, double *out);

/* Radius of the shrinking circle / sphere of the mean-curvature examples
 * (Sec. 4.2.2) from the phase volume V of ace_phase_volume: the radius of
 * the disc (d = 2, V = pi R^2) or ball (d = 3, V = 4/3 pi R^3) holding it,
 * and half the phase length (d = 1, V = 2 R).  Synchronous; *R is host
 * memory.  Errors as ace_phase_volume. */
int ace_equivalent_radius(ace_solver *s, double *R);

/* Copies the current field (total doubles, C order) to out. */
int ace_get_phi(ace_solver *s, double *out, int where);

/* Steps taken since the last ace_set_phi0. */
int64_t ace_step_count(const ace_solver *s);

/* Device pointer of the current field (valid until the next step). */
const double *ace_field_ptr(const ace_solver *s);

const char *ace_strerror(int status);

/* ---- reverse mode (adjoint of the time loop) ---------------------------- */

/* Gradient of a loss L(phi^T) through nsteps steps from phi0, given
 * lambdaT = dL/dphi^T.  Each step is phi^{n+1} = R(xi(phi^n)) with R the
 * root of the cubic, so the transposed step is
 *   mu      = lambda^{n+1} / (1 + h (3 (phi^{n+1})^2 - 1)),
 *   lambda^n = (1 - h (3 (phi^n)^2 - 1)) mu + kappa Lambda mu
 * (Lambda is symmetric: the D matrices of Sec. 2 are), and
 *   dL/dkappa = sum_n < mu, Lambda phi^n >.
 * Forward states are checkpointed every ckpt_every steps (>= 1) on the
 * device and each segment is recomputed during the reverse sweep.
 * Outputs: dphi0 (total doubles) and *deps2 = (dt/dx^2) dL/dkappa
 * (host double).  phi0, lambdaT and dphi0 live where `where` says.  The
 * handle's field afterwards holds phi^T.  Errors: ACE_E_NOMEM, ACE_E_ARG. */
int ace_adjoint(ace_solver *s, const double *phi0, int64_t nsteps,
                int64_t ckpt_every, const double *lambdaT, double *dphi0,
                double *deps2, int where);

/* The two halves of ace_adjoint, for callers that need phi^T before they can
 * form lambdaT (e.g. an autograd forward/backward pair).
 * ace_forward_ckpt sets phi^0 (where: ACE_HOST or ACE_DEVICE), advances
 * nsteps and keeps every ckpt_every-th state (steps 0, k, 2k, ...) in device
 * memory owned by the handle; the field then holds phi^T.
 * ace_backward consumes those checkpoints: given lambdaT = dL/dphi^T it
 * recomputes each segment and runs the transposed steps in reverse, writing
 * dphi0 and *deps2 (host).  Errors: ACE_E_STATE if no checkpoints exist or
 * the field was changed since ace_forward_ckpt. */
int ace_forward_ckpt(ace_solver *s, const double *phi0, int where, int64_t nsteps,
                     int64_t ckpt_every);  /* ACE_E_STATE under ACE_SCHEME_FEX */
int ace_backward(ace_solver *s, const double *lambdaT, double *dphi0, double *deps2,
                 int where);

/* Generation of the handle's checkpoints: 0 before the first
 * ace_forward_ckpt, then incremented by every successful ace_forward_ckpt.
 * A caller that keeps several forward passes on one handle (e.g. an
 * autograd graph with two of them) compares it with the value read after
 * its own forward to know whether ace_backward would use its checkpoints
 * or a later pass's.  Returns -1 for a NULL handle. */
int64_t ace_ckpt_generation(const ace_solver *s);

/* ---- mesoscopic form: populations of the DdQ(2d+1) lattice -------------- */

/* The regularized evolution equation of Sec. 2 before its summation over k:
 * 2d+1 populations per node (k = 0 at rest, k = 1..d moving along +axis
 * k-1, k = d+1..2d along -axis k-d-1; axis 0 is the slowest storage axis),
 * with equilibrium w_k phi, source -w_k f(phi), weights w_0 = 1 - 2 d w_1,
 * w_1 = omega1, and the non-equilibrium part regularized through the
 * first-order gradient of phi; s = omega1 / kappa.  Summing the populations
 * gives the FD step of ace_step (Sec. 2), so ace_pop_get_phi follows the
 * solver's field to rounding, while the handle holds 2 (2d+1) fields instead
 * of 2 and moves 16 (2d+1) bytes per node update instead of 16.
 * ace_pop_create takes the ace_create arguments plus omega1 in
 * (0, 1/(2d)] (0 selects the weights of the paper's experiments: 1/3, 1/5,
 * 1/6 for d = 1, 2, 3).  Errors as ace_create, ACE_E_ARG for omega1;
 * warning ACE_W_CONDITIONS as ace_create. */
typedef struct ace_pop ace_pop;
int ace_pop_create(int d, const int64_t N[], const double L[], const double R[], double eps,
                   double dt, int bc, double omega1, ace_pop **out);
int ace_pop_destroy(ace_pop *p);
/* Stored nodes per axis, node count, populations per node (2d+1), omega1,
 * s, and the device bytes the handle holds (any output may be NULL). */
int ace_pop_info(const ace_pop *p, int64_t M[3], int64_t *total, int *q, double *omega1,
                 double *s, int64_t *device_bytes);
int ace_pop_set_stream(ace_pop *p, void *hip_stream);
/* Kernel of ace_pop_step (every choice computes the same result bit for
 * bit): ACE_POP_DIRECT one thread per node, phi of the node and its
 * neighbours summed from their populations; ACE_POP_FUSED cache-line-
 * aligned tiles marching along axis 0 that sum phi of the tile and its ring
 * into LDS and write the new populations (16 (2d+1) bytes per node update);
 * ACE_POP_SPLIT a streaming pass writing phi = sum_k f_k, then the same
 * tiled update reading phi (16 (2d+1) + 16 bytes); ACE_POP_CARRY the same
 * tiled update, which also writes phi of the new populations (the sum over
 * k in the fixed order every moment here uses), so the next step reads phi
 * alone: the regularized update depends on the populations only through
 * phi (Sec. 2), and a step moves 8 (2d+1) + 16 bytes per node (one moment
 * pass after ace_pop_set_phi0 / ace_pop_set_populations or another kernel's
 * step; d >= 2, two more fields of device memory);
 * ACE_POP_AUTO: the carried form for d >= 2, direct for d = 1. */
#define ACE_POP_AUTO 0
#define ACE_POP_DIRECT 1
#define ACE_POP_FUSED 2
#define ACE_POP_SPLIT 3
#define ACE_POP_CARRY 4
int ace_pop_set_kernel(ace_pop *p, int kernel);
/* Populations at equilibrium f_k = w_k phi0 (phi0: total doubles, C order);
 * resets the step count.  ACE_E_NONFINITE for a non-finite host value. */
int ace_pop_set_phi0(ace_pop *p, const double *phi0, int where);
/* All populations, (2d+1) x total doubles, population-major. */
int ace_pop_set_populations(ace_pop *p, const double *f, int where);
int ace_pop_get_populations(const ace_pop *p, double *f, int where);
/* nsteps steps of the evolution equation (asynchronous on the stream). */
int ace_pop_step(ace_pop *p, int64_t nsteps);
/* phi = sum_k f_k (total doubles). */
int ace_pop_get_phi(ace_pop *p, double *phi, int where);
int64_t ace_pop_step_count(const ace_pop *p);

/* ---- batches of independent instances ----------------------------------- */

typedef struct ace_batch ace_batch;

/* One instance of a batch: the ace_create arguments. */
typedef struct {
    int d;
    int bc;
    int64_t N[3];
    double L[3];
    double R[3];
    double eps;
    double dt;
} ace_instance_desc;

/* Creates a batch of count instances (each validated as ace_create does;
 * status[i] receives each instance's status when status is not NULL).
 * Allocates one device arena for all fields.  Instances of one batch run in
 * persistent launches: each workgroup takes whole instances, one at a time,
 * from a queue ordered by decreasing cost, and runs all their steps (with
 * register-resident regions, the large 2D instances first in a kernel of
 * their own, then the rest; see ace_batch_set_region). */
int ace_batch_create(int count, const ace_instance_desc *desc,
                     ace_batch **out, int *status);
int ace_batch_destroy(ace_batch *b);
/* Stored nodes of instance i (M[0..2]) and its offset in doubles into the
 * arena (for device-side initialisation). */
int ace_batch_shape(const ace_batch *b, int i, int64_t M[3], int64_t *total,
                    int64_t *offset);
/* Stream of the batch's launches; switching waits for the old stream first
 * (as ace_set_stream). */
int ace_batch_set_stream(ace_batch *b, void *hip_stream);
/* Sets phi^0 of instance i (host or device pointer). */
int ace_batch_set_phi0(ace_batch *b, int i, const double *phi0, int where);
/* Sets every instance's phi^0 from one host array holding all instances
 * back to back in instance order (sum of totals doubles). */
int ace_batch_set_all(ace_batch *b, const double *phi0_all, int where);
/* Advances every instance by nsteps (asynchronous on the batch's stream). */
int ace_batch_step(ace_batch *b, int64_t nsteps);
/* Energy and max-norm of every instance (host arrays of count doubles). */
int ace_batch_monitor(ace_batch *b, double *E, double *maxn);
/* enable = 1 (default): each ace_batch_step replays a HIP graph holding the
 * queue reset and the persistent launches (captured once per step count);
 * 0: they are issued directly on the stream (e.g. for tools that do not
 * follow graph launches).  Results are identical either way. */
int ace_batch_set_graphs(ace_batch *b, int enable);
int ace_batch_get_phi(ace_batch *b, int i, double *out, int where);
int ace_batch_get_all(ace_batch *b, double *out_all, int where);
/* Instances with at most `limit` stored nodes are stepped entirely in LDS
 * (limit is capped at the LDS capacity, 8000 doubles); larger ones stream
 * through their two arena slots.  Results do not depend on the choice. */
int ace_batch_set_resident_limit(ace_batch *b, int64_t limit);
/* Steps per round (temporal-blocking depth, 1..8, default 4) of the 2D
 * instances too large for LDS, which advance over the regions of
 * ace_batch_set_region with a ring of `depth` nodes recomputed.  Results do
 * not depend on the choice.  Error: ACE_E_ARG outside 1..8. */
int ace_batch_set_depth(ace_batch *b, int depth);
/* Region of the 2D instances too large for LDS: rows = 0 (default) the
 * 32 x 64 regions kept in LDS level by level; 32 or 64 the register-resident
 * regions of that many rows by 64 columns (each thread two or four rows of a
 * column; nodes outside the instance are its boundary images), the region
 * shape of ace_set_region2d, stepped by a kernel of their own launched before
 * the one for the other instances.  Results do not depend on the choice.
 * Error: ACE_E_ARG for other values. */
int ace_batch_set_region(ace_batch *b, int rows);
/* Times one batch step of trial_steps steps on the current fields (which are
 * restored): first for every region (0, 32, 64) and depth 2..6 at the
 * current resident limit, then for several resident limits at the fastest
 * pair.  Keeps the fastest and writes a JSON record of the timings into json
 * (capacity cap, may be NULL). */
int ace_batch_autotune(ace_batch *b, int64_t trial_steps, char *json, size_t cap);

/* ---- autotuner ------------------------------------------------------------ */

/* Times each kernel choice on the handle's problem for trial_steps steps
 * from the current field: the one-thread-per-node, LDS-resident (small
 * fields) and marching kernels, the 3D blocked kernels (the two-step kernel
 * and every depth and region shape of ace_set_region3d) at several plane
 * chunks and as a persistent grid, and the 2D blocked kernels (every region
 * of ace_set_region2d) at depths 1-6, 8, 10, 12.  Each
 * trial is run once untimed and then timed; a trial shorter than 2 ms is
 * lengthened to about 2 ms (at most 2^20 steps), so that small fields are
 * timed in the steady state of a long run.  The trials time ace_step only.
 * Keeps the fastest as the ACE_KERNEL_AUTO choice, restores the field, and
 * writes a one-line JSON record of the timings into json (capacity cap
 * bytes, may be NULL).  If the environment variable ACE_AUTOTUNE_CACHE names
 * a file, the choice is appended there (one JSON object per line: d, bc, M,
 * kernel, zchunk, depth2, tb3 (the 3D variant, -1 for the two-step
 * kernel), tb2 (the 2D variant, -1 for the LDS-plane kernel), ms_per_step)
 * and later handles of the same
 * (d, bc, shape) reuse it. */
int ace_autotune(ace_solver *s, int64_t trial_steps, char *json, size_t cap);

/* Diagnostics: if the environment variable ACE_LOG is set, the library
 * prints one "[ace]" line on stderr per HIP error, handle creation (derived
 * parameters, Newton count), graph capture (launch configuration) and
 * autotuner choice. */

/* Library version string. */
const char *ace_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ACE_H */
