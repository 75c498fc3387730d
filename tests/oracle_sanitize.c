/*
 * Exercises the C part of the oracle (oracle/wilson_oracle.c) under
 * AddressSanitizer and UndefinedBehaviorSanitizer: every entry point on small
 * lattices, ragged extents included, with seeded inputs, and two identities
 * so that the run computes something checkable:
 *   <phi, D psi> = <D^H phi, psi>,   A psi = D^H (D psi),
 * and the site-sampled forms equal the full ones at the sampled sites.
 * Exit status 0 when every check holds; a sanitizer report aborts the run.
 * Test infrastructure only (built and run by tests/test_oracle_sanitizers.py).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;

void oracle_gamma(int mu, cplx *out16);
void oracle_neighbors(const int32_t L[4], int32_t *out);
void oracle_apply_D(const int32_t L[4], const cplx *U, double kappa, const cplx *psi, cplx *out, int32_t m,
                    int32_t dagger);
int oracle_apply_A(const int32_t L[4], const cplx *U, double kappa, const cplx *psi, cplx *out, int32_t m);
void oracle_apply_D_sites(const int32_t L[4], const cplx *U, double kappa, const cplx *psi, int32_t m,
                          int32_t dagger, const int64_t *sites, int64_t nsites, cplx *out);
int oracle_apply_A_sites(const int32_t L[4], const cplx *U, double kappa, const cplx *psi, int32_t m,
                         const int64_t *sites, int64_t nsites, cplx *out);
void oracle_link_grad(const int32_t L[4], double kappa, const cplx *phi, const cplx *psi, int32_t m,
                      cplx *out);
int oracle_max_threads(void);

static uint64_t state;
static double uniform(void) {
    /* 64-bit linear congruential generator (Knuth's MMIX constants) */
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(state >> 11) / 9007199254740992.0 - 0.5;
}
static void fill(cplx *a, size_t n) {
    for (size_t i = 0; i < n; ++i) a[i] = uniform() + I * uniform();
}
static cplx dot(const cplx *a, const cplx *b, size_t n) {
    cplx s = 0;
    for (size_t i = 0; i < n; ++i) s += conj(a[i]) * b[i];
    return s;
}
static double maxdiff(const cplx *a, const cplx *b, size_t n) {
    double d = 0.0, s = 0.0;
    for (size_t i = 0; i < n; ++i) {
        d = fmax(d, cabs(a[i] - b[i]));
        s = fmax(s, cabs(b[i]));
    }
    return s > 0 ? d / s : d;
}

static int run(const int32_t L[4], int32_t m, uint64_t seed) {
    state = seed;
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    const size_t nf = (size_t)V * 12 * m, nu = (size_t)V * 36;
    cplx *U = malloc(sizeof(cplx) * nu), *psi = malloc(sizeof(cplx) * nf), *phi = malloc(sizeof(cplx) * nf);
    cplx *Dpsi = malloc(sizeof(cplx) * nf), *Dhphi = malloc(sizeof(cplx) * nf), *A1 = malloc(sizeof(cplx) * nf);
    cplx *A2 = malloc(sizeof(cplx) * nf), *G = malloc(sizeof(cplx) * nu), *g16 = malloc(sizeof(cplx) * 16);
    int32_t *nb = malloc(sizeof(int32_t) * (size_t)V * 8);
    int fails = 0;
    fill(U, nu);
    fill(psi, nf);
    fill(phi, nf);
    for (int mu = 0; mu < 4; ++mu) oracle_gamma(mu, g16);
    oracle_neighbors(L, nb);
    for (int64_t x = 0; x < V * 8; ++x)
        if (nb[x] < 0 || nb[x] >= V) ++fails;
    oracle_apply_D(L, U, 0.13, psi, Dpsi, m, 0);
    oracle_apply_D(L, U, 0.13, phi, Dhphi, m, 1);
    const cplx l = dot(phi, Dpsi, nf), r = dot(Dhphi, psi, nf);
    if (cabs(l - r) > 1e-12 * cabs(l)) ++fails;
    if (oracle_apply_A(L, U, 0.13, psi, A1, m) != 0) ++fails;
    oracle_apply_D(L, U, 0.13, Dpsi, A2, m, 1);
    if (maxdiff(A1, A2, nf) > 1e-14) ++fails;
    int64_t sites[3] = {0, V / 2, V - 1};
    cplx *Ds = malloc(sizeof(cplx) * 3 * 12 * m), *As = malloc(sizeof(cplx) * 3 * 12 * m);
    oracle_apply_D_sites(L, U, 0.13, psi, m, 0, sites, 3, Ds);
    if (oracle_apply_A_sites(L, U, 0.13, psi, m, sites, 3, As) != 0) ++fails;
    for (int k = 0; k < 3; ++k) {
        if (maxdiff(Ds + (size_t)k * 12 * m, Dpsi + (size_t)sites[k] * 12 * m, (size_t)12 * m) > 1e-14) ++fails;
        if (maxdiff(As + (size_t)k * 12 * m, A1 + (size_t)sites[k] * 12 * m, (size_t)12 * m) > 1e-14) ++fails;
    }
    oracle_link_grad(L, 0.13, phi, psi, m, G);
    printf("L = %d %d %d %d, m = %d: %d failed checks\n", L[0], L[1], L[2], L[3], m, fails);
    free(U); free(psi); free(phi); free(Dpsi); free(Dhphi); free(A1); free(A2); free(G); free(g16);
    free(nb); free(Ds); free(As);
    return fails;
}

int main(void) {
    const int32_t lat[4][4] = {{2, 2, 2, 2}, {3, 4, 5, 2}, {4, 3, 2, 5}, {2, 3, 3, 4}};
    const int32_t ms[4] = {1, 3, 2, 4};
    int fails = 0;
    printf("threads %d\n", oracle_max_threads());
    for (int k = 0; k < 4; ++k) fails += run(lat[k], ms[k], 1205u + (uint64_t)k);
    return fails ? 1 : 0;
}
