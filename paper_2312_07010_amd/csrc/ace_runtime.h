// Host-side pieces shared by the solver and batch runtimes.
#pragma once

#include <stdint.h>

#include "ace_internal.h"

namespace ace {

// Validated problem of one handle or batch instance (Sec. 2 notation).
struct Problem {
    int d, bc;
    int64_t N[3], M[3], total;
    double L[3], R[3];
    double dx, dt, eps, kappa, h;
    int nit;
    int start2;  // second-order start of the root iteration
    int cond_ok;
    int scheme;  // ACE_SCHEME_*
};

// True if the environment variable ACE_LOG is set: the library then reports
// HIP errors, handle parameters, graph captures and autotuner choices on
// stderr, one "[ace]" line each.
bool log_enabled();
int hip_status(hipError_t e);
int64_t nodes_per_axis(int64_t N, int bc);
// Newton steps that bring the root iteration (first- or second-order start)
// within 2^-60 of the root for every |xi| in (0, 1].
int newton_iters_for(double h, int start2);
// ACE_OK, ACE_W_CONDITIONS or a negative error.
int derive(int d, const int64_t *N, const double *L, const double *R, double eps, double dt,
           int bc, Problem &p);
Shape shape_of(const Problem &p);
StepCoef coef_of(const Problem &p);
// E = dxd (bulk + cg grad) with dxd = dx^d and cg = kappa / (2 dt).
void energy_coefs(const Problem &p, double *dxd, double *cg);
double energy_from(const Problem &p, const double *trip);
// (Re)allocates *ptr to hold at least need doubles of device memory.
int grow(double **ptr, int64_t *cap, int64_t need);

}  // namespace ace
