/*
 * CPU oracle for the RLB-MIE-FD scheme of Chen, Liu, Chai and Shi,
 * "Regularized lattice Boltzmann method based maximum principle and energy
 * stability preserving finite-difference scheme for the Allen-Cahn equation"
 * (arXiv 2312.07010).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or constant with the GPU library, and the GPU
 * library never calls it.
 *
 * Arithmetic is IEEE double (compile with -ffp-contract=off, no fast-math)
 * except the root of the pointwise cubic, which is computed in x87 extended
 * precision (long double) and rounded once to double.
 *
 * Notation (paper): d = dimension, N = cells per axis, Delta x = X/N,
 * kappa = omega_1/s = eps^2 Delta t / Delta x^2 (the paper's lattice
 * epsilon, renamed here so it does not clash with the interface width eps),
 * h = Delta t / 2, f(phi) = phi^3 - phi.
 *
 * Readings where the paper is silent or garbled:
 *  - periodic BC stores N unique nodes i = 0..N-1 (period X); the printed
 *    circulant of size N+1 would duplicate the node at x = R;
 *  - homogeneous Neumann stores N+2 nodes at x = L + (i - 1/2) Delta x, the
 *    size of the printed matrix with -1 corners (mirror neighbour = self);
 *  - homogeneous Dirichlet stores N-1 nodes at x = L + i Delta x,
 *    i = 1..N-1 (stored index i-1); the two wall nodes hold 0 and are not
 *    stored;
 *  - the d = 3 operator is the isotropic 7-point sum I(x)I(x)D + I(x)D(x)I +
 *    D(x)I(x)I (the printed first and last terms coincide).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Loops over fewer nodes than this run on one thread: a parallel region per
 * step of a small field costs more than it saves.  Results do not depend on
 * the thread count. */
#define ORACLE_PAR_MIN 16384

#define BC_HN 0
#define BC_HD 1
#define BC_P 2

/* ---------------------------------------------------------------------- */
/* Layout (Sec. 2: grid function space and node positions)                */
/* ---------------------------------------------------------------------- */

/* Stored nodes per axis for N cells under boundary condition bc.         */
long oracle_nodes_per_axis(long N, int bc)
{
    if (bc == BC_HN) return N + 2;
    if (bc == BC_HD) return N - 1;
    return N; /* periodic */
}

/* Coordinate of stored node i on an axis starting at L with spacing dx.  */
double oracle_node_coord(int bc, double L, double dx, long i)
{
    if (bc == BC_HN) return L + ((double)i - 0.5) * dx;
    if (bc == BC_HD) return L + (double)(i + 1) * dx;
    return L + (double)i * dx;
}

/* kappa = eps^2 dt / dx^2: the map between the diffusion coefficient and the
 * lattice parameter omega_1/s (Sec. 2, below the vector form).           */
double oracle_kappa(double eps, double dt, double dx)
{
    return eps * eps * dt / (dx * dx);
}

/* ---------------------------------------------------------------------- */
/* Pointwise cubic (Sec. 3.2, Remark 1)                                    */
/* ---------------------------------------------------------------------- */

/* Unique real root theta of  theta + h (theta^3 - theta) = xi  for
 * 0 < h < 1 (0 < dt < 2).  The root map is odd in xi, so the root is found
 * for |xi| and the sign restored.  Where the root is known exactly (xi = 0,
 * |xi| = 1) it is returned directly.  Otherwise the closed form of Remark 1,
 *     theta0 = (zeta + sqrt(zeta^2 - D^3))^(1/3)
 *              + D (zeta + sqrt(zeta^2 - D^3))^(-1/3),
 *     zeta = xi/dt,  D = (dt - 2)/(3 dt),
 * is evaluated in long double and then polished by Newton's method on the
 * cubic in long double until it stops moving (the closed form cancels
 * badly for small |xi|), and the result is rounded once to double.        */
double oracle_root(double xi, double h)
{
    if (xi == 0.0) return xi; /* keeps the sign of a signed zero */
    if (xi == 1.0 || xi == -1.0) return xi;
    const long double a = fabsl((long double)xi);
    const long double H = (long double)h;
    const long double dt = 2.0L * H;
    const long double zeta = a / dt;
    const long double D = (dt - 2.0L) / (3.0L * dt);
    const long double s = zeta + sqrtl(zeta * zeta - D * D * D);
    const long double A = cbrtl(s);
    long double th = A + D / A;
    if (!(th > 0.0L) || !isfinite((double)th)) th = a; /* safe start */
    long double prev_step = INFINITY;
    for (int it = 0; it < 200; ++it) {
        const long double p = th + H * (th * th * th - th) - a;
        const long double dp = 1.0L + H * (3.0L * th * th - 1.0L);
        const long double step = p / dp;
        const long double nxt = th - step;
        if (nxt == th) break;
        if (fabsl(step) >= prev_step) break; /* rounding-level noise */
        prev_step = fabsl(step);
        th = nxt;
    }
    const double r = (double)th;
    return xi < 0 ? -r : r;
}

/* ---------------------------------------------------------------------- */
/* One step of the scheme (Sec. 2, pointwise form IE-FD and vector form)   */
/* ---------------------------------------------------------------------- */

static void strides(int d, const long *M, long *st)
{
    st[d - 1] = 1;
    for (int k = d - 2; k >= 0; --k) st[k] = st[k + 1] * M[k + 1];
}

/* Value of the neighbour of flat node idx one step along axis k in
 * direction dir (-1 or +1).  Out-of-range neighbours follow the boundary
 * rows of the paper's D matrices: Neumann mirrors the node itself (row
 * (-1, 1)), Dirichlet reads the zero wall value, periodic wraps.          */
static double neighbour(const double *phi, int d, const long *M,
                        const long *st, int bc, long idx, int k, int dir)
{
    (void)d;
    const long c = (idx / st[k]) % M[k];
    const long cn = c + dir;
    if (cn >= 0 && cn < M[k]) return phi[idx + dir * st[k]];
    if (bc == BC_HN) return phi[idx];
    if (bc == BC_HD) return 0.0;
    /* periodic wrap */
    const long cw = (cn < 0) ? M[k] - 1 : 0;
    return phi[idx + (cw - c) * st[k]];
}

/* Explicit part of node idx:
 *   xi = phi + kappa * sum_k (phi_{+k} + phi_{-k} - 2 phi) - h f(phi).    */
static double explicit_part(const double *phi, int d, const long *M,
                            const long *st, int bc, double kappa, double h,
                            long idx)
{
    const double p = phi[idx];
    double lap = 0.0;
    for (int k = 0; k < d; ++k) {
        const double lo = neighbour(phi, d, M, st, bc, idx, k, -1);
        const double hi = neighbour(phi, d, M, st, bc, idx, k, +1);
        lap = lap + (hi + lo - 2.0 * p);
    }
    const double fp = p * p * p - p;
    return p + kappa * lap - h * fp;
}

long oracle_total(int d, const long *M)
{
    long n = 1;
    for (int k = 0; k < d; ++k) n *= M[k];
    return n;
}

/* Explicit parts of every node (used by the pins on the stencil alone).  */
void oracle_xi(int d, const long *M, int bc, double kappa, double h,
               const double *phi, double *xi)
{
    long st[3];
    strides(d, M, st);
    const long n = oracle_total(d, M);
#pragma omp parallel for schedule(static) if (n >= ORACLE_PAR_MIN)
    for (long i = 0; i < n; ++i)
        xi[i] = explicit_part(phi, d, M, st, bc, kappa, h, i);
}

/* phi^{n+1} from phi^n for every stored node.  out must not alias phi.  */
void oracle_step(int d, const long *M, int bc, double kappa, double h,
                 const double *phi, double *out)
{
    long st[3];
    strides(d, M, st);
    const long n = oracle_total(d, M);
#pragma omp parallel for schedule(static) if (n >= ORACLE_PAR_MIN)
    for (long i = 0; i < n; ++i)
        out[i] = oracle_root(explicit_part(phi, d, M, st, bc, kappa, h, i), h);
}

/* The fully explicit comparison scheme of Sec. 3.3, Remark 2 (FEX-FD):
 * forward Euler in time with the same central Laplacian, all of f explicit,
 *   phi^{n+1} = phi + kappa * sum_k (phi_{+k} + phi_{-k} - 2 phi) - dt f(phi).
 * (The paper states only its step condition dt <= (1 - 2 d kappa)/2; this
 * is the standard scheme that condition belongs to.)                       */
void oracle_step_fex(int d, const long *M, int bc, double kappa, double dt,
                     const double *phi, double *out)
{
    long st[3];
    strides(d, M, st);
    const long n = oracle_total(d, M);
#pragma omp parallel for schedule(static) if (n >= ORACLE_PAR_MIN)
    for (long i = 0; i < n; ++i) {
        const double p = phi[i];
        double lap = 0.0;
        for (int k = 0; k < d; ++k) {
            const double lo = neighbour(phi, d, M, st, bc, i, k, -1);
            const double hi = neighbour(phi, d, M, st, bc, i, k, +1);
            lap = lap + (hi + lo - 2.0 * p);
        }
        const double fp = p * p * p - p;
        out[i] = p + kappa * lap - dt * fp;
    }
}

/* ---------------------------------------------------------------------- */
/* Monitors (Sec. 3.2 maximum norm, Sec. 3.3 Theorem 3 discrete energy)    */
/* ---------------------------------------------------------------------- */

typedef struct { double s, c; } neumaier_t;

static void nsum_add(neumaier_t *a, double x)
{
    const double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_get(const neumaier_t *a) { return a->s + a->c; }

/* Sum over stored nodes of (phi^2 - 1)^2 / 4.                            */
double oracle_bulk_sum(long n, const double *phi)
{
    neumaier_t acc = {0, 0};
    for (long i = 0; i < n; ++i) {
        const double q = phi[i] * phi[i] - 1.0;
        nsum_add(&acc, 0.25 * q * q);
    }
    return nsum_get(&acc);
}

/* G = -Phi^T Lambda Phi with Lambda = dx^2 Lambda_dx, written as the sum
 * over lattice edges of squared differences: each axis-aligned pair of
 * neighbouring stored nodes once, plus for Dirichlet the edge from each end
 * node to its zero wall node, plus for periodic the wrap edge of each line
 * (its two ends).  Neumann has no boundary edge: its corner -1 rows give
 * exactly the interior edge sum.                                          */
double oracle_grad_sum(int d, const long *M, int bc, const double *phi)
{
    long st[3];
    strides(d, M, st);
    const long n = oracle_total(d, M);
    neumaier_t acc = {0, 0};
    for (long i = 0; i < n; ++i) {
        for (int k = 0; k < d; ++k) {
            const long c = (i / st[k]) % M[k];
            if (c + 1 < M[k]) {
                const double df = phi[i + st[k]] - phi[i];
                nsum_add(&acc, df * df);
            } else if (bc == BC_P) {
                /* wrap edge between the last and the first node */
                const double df = phi[i - (M[k] - 1) * st[k]] - phi[i];
                if (M[k] > 1) nsum_add(&acc, df * df);
            } else if (bc == BC_HD) {
                nsum_add(&acc, phi[i] * phi[i]); /* edge to right wall */
            }
            if (bc == BC_HD && c == 0)
                nsum_add(&acc, phi[i] * phi[i]); /* edge to left wall */
        }
    }
    return nsum_get(&acc);
}

/* E = dx^d [ sum (phi^2-1)^2/4 - kappa/(2 dt) Phi^T Lambda Phi ].        */
double oracle_energy(int d, const long *M, int bc, double kappa, double dt,
                     double dx, const double *phi)
{
    const long n = oracle_total(d, M);
    const double bulk = oracle_bulk_sum(n, phi);
    const double grad = oracle_grad_sum(d, M, bc, phi);
    return pow(dx, d) * (bulk + kappa / (2.0 * dt) * grad);
}

double oracle_maxnorm(long n, const double *phi)
{
    double m = 0.0;
    for (long i = 0; i < n; ++i) {
        const double a = fabs(phi[i]);
        if (a > m || a != a) m = a;
        if (m != m) return m;
    }
    return m;
}

/* ---------------------------------------------------------------------- */
/* Time loop (Sec. 2, vector form for 0 <= n <= N_t - 1)                   */
/* ---------------------------------------------------------------------- */

/* Advance phi in place by nsteps.  If every > 0, E[j] and maxn[j] receive
 * the monitors at steps 0, every, 2*every, ... <= nsteps (arrays of length
 * nsteps/every + 1).  Returns 0, or -1 when scratch memory is missing.    */
int oracle_run_scheme(int d, const long *M, int bc, double kappa, double dt,
                      double dx, double *phi, long nsteps, long every, double *E,
                      double *maxn, int scheme);

int oracle_run(int d, const long *M, int bc, double kappa, double dt,
               double dx, double *phi, long nsteps, long every, double *E,
               double *maxn)
{
    return oracle_run_scheme(d, M, bc, kappa, dt, dx, phi, nsteps, every, E, maxn, 0);
}

/* scheme 0: the RLB-MIE-FD step; scheme 1: FEX-FD (Remark 2).           */
int oracle_run_scheme(int d, const long *M, int bc, double kappa, double dt,
                      double dx, double *phi, long nsteps, long every, double *E,
                      double *maxn, int scheme)
{
    const long n = oracle_total(d, M);
    const double h = 0.5 * dt;
    double *tmp = (double *)malloc((size_t)n * sizeof(double));
    if (!tmp) return -1;
    double *cur = phi, *nxt = tmp;
    long j = 0;
    for (long s = 0; s <= nsteps; ++s) {
        if (every > 0 && s % every == 0) {
            E[j] = oracle_energy(d, M, bc, kappa, dt, dx, cur);
            maxn[j] = oracle_maxnorm(n, cur);
            ++j;
        }
        if (s == nsteps) break;
        if (scheme == 1) oracle_step_fex(d, M, bc, kappa, dt, cur, nxt);
        else oracle_step(d, M, bc, kappa, h, cur, nxt);
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != phi) memcpy(phi, cur, (size_t)n * sizeof(double));
    free(tmp);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Reverse-mode derivative of the time loop                                */
/* ---------------------------------------------------------------------- */

/* Given lambdaT = dL/dphi^{nsteps}, returns dphi0 = dL/dphi^0 and
 * *dkappa = dL/dkappa (the caller multiplies by dt/dx^2 for dL/d(eps^2)).
 *
 * Each step is phi^{n+1}_i = R(xi_i(phi^n)) with R the root of the cubic.
 * Differentiating the cubic gives dR/dxi = 1 / (1 + h (3 R^2 - 1)).  The
 * explicit part has Jacobian diag(1 - h (3 phi^2 - 1)) + kappa Lambda, and
 * Lambda is symmetric (Sec. 2, the D matrices are symmetric), so the
 * transposed step applies the same stencil.  dxi/dkappa = Lambda phi^n.
 * All forward states are kept in memory (no recomputation).               */
int oracle_adjoint(int d, const long *M, int bc, double kappa, double dt,
                   const double *phi0, long nsteps, const double *lambdaT,
                   double *dphi0, double *dkappa)
{
    const long n = oracle_total(d, M);
    const double h = 0.5 * dt;
    long st[3];
    strides(d, M, st);
    double *states = (double *)malloc((size_t)n * (size_t)(nsteps + 1) * sizeof(double));
    double *lam = (double *)malloc((size_t)n * sizeof(double));
    double *mu = (double *)malloc((size_t)n * sizeof(double));
    double *lapf = (double *)malloc((size_t)n * sizeof(double));
    if (!states || !lam || !mu || !lapf) {
        free(states); free(lam); free(mu); free(lapf);
        return -1;
    }
    memcpy(states, phi0, (size_t)n * sizeof(double));
    for (long s = 0; s < nsteps; ++s)
        oracle_step(d, M, bc, kappa, h, states + (size_t)s * n,
                    states + (size_t)(s + 1) * n);
    memcpy(lam, lambdaT, (size_t)n * sizeof(double));
    neumaier_t gk = {0, 0};
    for (long s = nsteps - 1; s >= 0; --s) {
        const double *pn = states + (size_t)s * n;
        const double *pn1 = states + (size_t)(s + 1) * n;
        for (long i = 0; i < n; ++i)
            mu[i] = lam[i] / (1.0 + h * (3.0 * pn1[i] * pn1[i] - 1.0));
        for (long i = 0; i < n; ++i) {
            /* (Lambda mu)_i and (Lambda phi^n)_i with the same BC rows */
            double lm = 0.0, lp = 0.0;
            for (int k = 0; k < d; ++k) {
                lm += neighbour(mu, d, M, st, bc, i, k, -1) +
                      neighbour(mu, d, M, st, bc, i, k, +1) - 2.0 * mu[i];
                lp += neighbour(pn, d, M, st, bc, i, k, -1) +
                      neighbour(pn, d, M, st, bc, i, k, +1) - 2.0 * pn[i];
            }
            lapf[i] = (1.0 - h * (3.0 * pn[i] * pn[i] - 1.0)) * mu[i] + kappa * lm;
            nsum_add(&gk, mu[i] * lp);
        }
        memcpy(lam, lapf, (size_t)n * sizeof(double));
    }
    memcpy(dphi0, lam, (size_t)n * sizeof(double));
    *dkappa = nsum_get(&gk);
    free(states); free(lam); free(mu); free(lapf);
    return 0;
}

/* Roots for an array of explicit parts (used by the pins on the root).   */
void oracle_root_array(long n, const double *xi, double h, double *out)
{
#pragma omp parallel for schedule(static) if (n >= ORACLE_PAR_MIN)
    for (long i = 0; i < n; ++i) out[i] = oracle_root(xi[i], h);
}

/* Volume of the phase phi > 0, measured smoothly as dx^d sum (1 + phi)/2
 * (the tanh profile across the interface is odd, so this equals the volume
 * enclosed by the zero level set up to curvature corrections).  Used for the
 * equivalent radius in the mean-curvature examples of Sec. 4.2.2.         */
double oracle_phase_volume(int d, const long *M, double dx, const double *phi)
{
    const long n = oracle_total(d, M);
    neumaier_t acc = {0, 0};
    for (long i = 0; i < n; ++i) nsum_add(&acc, 0.5 * (1.0 + phi[i]));
    return pow(dx, d) * nsum_get(&acc);
}

/* ---------------------------------------------------------------------- */
/* Mesoscopic form (Sec. 2): populations of the DdQ(2d+1) lattice          */
/* ---------------------------------------------------------------------- */
/*
 * Population k = 0 rests; k = 1..d moves along +axis (k-1) and k = d+1..2d
 * along -axis (k-d-1), with axis 0 the slowest storage axis (the paper's
 * x_1).  Velocities c_k = +-c e, c = dx/dt.  Weights w_0 = 1 - 2 d w_1 and
 * w_1 = ... = w_2d (Sec. 2, moment conditions).  The q = 2d+1 arrays are
 * stored one after another: f[k * n + i].
 */

/* phi = sum_k f_k, the zeroth moment.                                     */
void oracle_pop_moment(int d, const long *M, const double *f, double *phi)
{
    const long n = oracle_total(d, M);
    const int q = 2 * d + 1;
#pragma omp parallel for schedule(static) if (n >= ORACLE_PAR_MIN)
    for (long i = 0; i < n; ++i) {
        double p = 0.0;
        for (int k = 0; k < q; ++k) p = p + f[k * n + i];
        phi[i] = p;
    }
}

/* Equilibrium populations f_k = w_k phi (Sec. 2, equilibrium distribution). */
void oracle_pop_equilibrium(int d, const long *M, double omega1, const double *phi,
                            double *f)
{
    const long n = oracle_total(d, M);
    const double w0 = 1.0 - 2.0 * d * omega1;
    for (long i = 0; i < n; ++i) {
        f[i] = w0 * phi[i];
        for (int k = 1; k <= 2 * d; ++k) f[k * n + i] = omega1 * phi[i];
    }
}

/* One step of the regularized evolution equation of Sec. 2 (the RLB form
 * before summation), taken in the paper's order:
 *   1. phi = sum_k f_k;
 *   2. for each population, the right-hand side
 *        RHS_k(x) = f_k^eq(x - c_k dt) + s_A w_k c_k . Pi^ne(x - c_k dt)
 *                   + (dt/2) F_k(x, t),
 *      with f_k^eq = w_k phi, F_k = -w_k f(phi), s_A = (1 - s)/c_s^2,
 *      c_s^2 = 2 w_1 c^2, Pi^ne = -dt c_s^2 grad(phi)/s, and the gradient at
 *      x - c_k dt by the first-order difference between that node and x;
 *      out-of-range nodes take the boundary condition's value (as in the
 *      D matrices);
 *   3. the left-hand side summed over k is phi(t+dt) + (dt/2) f(phi(t+dt)),
 *      so phi(t+dt) is the root of the pointwise cubic for xi = sum_k RHS_k;
 *   4. f_k(x, t+dt) = RHS_k + (dt/2) F_k(x, t+dt).                        */
void oracle_pop_step(int d, const long *M, int bc, double omega1, double s,
                     double dt, double dx, const double *f, double *fout)
{
    const long n = oracle_total(d, M);
    const int q = 2 * d + 1;
    long st[3];
    strides(d, M, st);
    double *phi = (double *)malloc(sizeof(double) * (size_t)n);
    oracle_pop_moment(d, M, f, phi);
    const double c = dx / dt;
    const double cs2 = 2.0 * omega1 * c * c;
    const double sA = (1.0 - s) / cs2;
    const double h = 0.5 * dt;
    const double w0 = 1.0 - 2.0 * d * omega1;
#pragma omp parallel for schedule(static) if (n >= ORACLE_PAR_MIN)
    for (long i = 0; i < n; ++i) {
        double rhs[7];
        const double p = phi[i];
        const double fp = p * p * p - p;
        rhs[0] = w0 * p + h * (w0 * (-fp));
        for (int a = 0; a < d; ++a) {
            /* k = 1 + a: c_k = +c e_a, from x - e_a dx */
            const double lo = neighbour(phi, d, M, st, bc, i, a, -1);
            const double pim = -dt * cs2 * ((p - lo) / dx) / s;
            rhs[1 + a] = omega1 * lo + sA * omega1 * (c * pim) + h * (omega1 * (-fp));
            /* k = 1 + d + a: c_k = -c e_a, from x + e_a dx */
            const double hi = neighbour(phi, d, M, st, bc, i, a, +1);
            const double pip = -dt * cs2 * ((hi - p) / dx) / s;
            rhs[1 + d + a] = omega1 * hi + sA * omega1 * (-c * pip) + h * (omega1 * (-fp));
        }
        double xi = 0.0;
        for (int k = 0; k < q; ++k) xi = xi + rhs[k];
        const double th = oracle_root(xi, h);
        const double ft = th * th * th - th;
        for (int k = 0; k < q; ++k) {
            const double w = (k == 0) ? w0 : omega1;
            fout[k * n + i] = rhs[k] + h * (w * (-ft));
        }
    }
    free(phi);
}

/* nsteps steps (ping-pong inside; f is overwritten with the result).     */
void oracle_pop_run(int d, const long *M, int bc, double omega1, double s, double dt,
                    double dx, double *f, long nsteps)
{
    const long n = oracle_total(d, M) * (2 * d + 1);
    double *g = (double *)malloc(sizeof(double) * (size_t)n);
    for (long t = 0; t < nsteps; ++t) {
        oracle_pop_step(d, M, bc, omega1, s, dt, dx, f, g);
        memcpy(f, g, sizeof(double) * (size_t)n);
    }
    free(g);
}

/* Threads the parallel loops above use (for timing the CPU baseline only;
 * results do not depend on it, since every parallel loop is a pointwise map
 * and the sums run serially). Returns the previous maximum. */
int oracle_set_threads(int n)
{
    int prev = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return prev;
}
