/*
 * Uses the library through its C ABI alone (no Python, no torch): a 2D
 * Neumann problem of n x n stored nodes read from a binary file of doubles,
 * `steps` steps of the scheme, then the field, the discrete energy and the
 * max-norm written out.  Also exercises the population form on the same
 * field.  Usage: ace_c_demo <n-cells> <eps> <dt> <steps> <in.bin> <out.bin>
 * (<in.bin> holds (n+2)^2 doubles; <out.bin> receives the field, then E and
 * the max-norm, then the population form's zeroth moment).
 */
#include <stdio.h>
#include <stdlib.h>

#include "ace.h"

static int check(int st, const char *what)
{
    if (st < 0) {
        fprintf(stderr, "%s: %s (%d)\n", what, ace_strerror(st), st);
        exit(1);
    }
    return st;
}

int main(int argc, char **argv)
{
    if (argc != 7) {
        fprintf(stderr, "usage: %s n eps dt steps in.bin out.bin\n", argv[0]);
        return 2;
    }
    const int64_t N[2] = {atoll(argv[1]), atoll(argv[1])};
    const double L[2] = {0.0, 0.0}, R[2] = {1.0, 1.0};
    const double eps = atof(argv[2]), dt = atof(argv[3]);
    const int64_t steps = atoll(argv[4]);
    ace_solver *s = NULL;
    check(ace_create(2, N, L, R, eps, dt, ACE_BC_HN, &s), "ace_create");
    int64_t M[3], total = 0;
    check(ace_shape(s, M, &total), "ace_shape");
    double *phi = (double *)malloc(sizeof(double) * (size_t)(total + 2));
    FILE *f = fopen(argv[5], "rb");
    if (!f || fread(phi, sizeof(double), (size_t)total, f) != (size_t)total) {
        fprintf(stderr, "cannot read %s\n", argv[5]);
        return 1;
    }
    fclose(f);
    check(ace_set_phi0(s, phi, ACE_HOST), "ace_set_phi0");
    check(ace_step(s, steps), "ace_step");
    check(ace_get_phi(s, phi, ACE_HOST), "ace_get_phi");
    check(ace_energy(s, &phi[total]), "ace_energy");
    check(ace_maxnorm(s, &phi[total + 1]), "ace_maxnorm");
    check(ace_destroy(s), "ace_destroy");

    ace_pop *p = NULL;
    check(ace_pop_create(2, N, L, R, eps, dt, ACE_BC_HN, 0.0, &p), "ace_pop_create");
    double *phi0 = (double *)malloc(sizeof(double) * (size_t)total);
    f = fopen(argv[5], "rb");
    if (!f || fread(phi0, sizeof(double), (size_t)total, f) != (size_t)total) return 1;
    fclose(f);
    check(ace_pop_set_phi0(p, phi0, ACE_HOST), "ace_pop_set_phi0");
    check(ace_pop_step(p, steps), "ace_pop_step");
    check(ace_pop_get_phi(p, phi0, ACE_HOST), "ace_pop_get_phi");
    check(ace_pop_destroy(p), "ace_pop_destroy");

    f = fopen(argv[6], "wb");
    if (!f) return 1;
    fwrite(phi, sizeof(double), (size_t)(total + 2), f);
    fwrite(phi0, sizeof(double), (size_t)total, f);
    fclose(f);
    printf("%s: %lld x %lld nodes, %lld steps, E = %.15e, max-norm = %.15e\n", ace_version(),
           (long long)M[0], (long long)M[1], (long long)steps, phi[total], phi[total + 1]);
    free(phi);
    free(phi0);
    return 0;
}
