/*
 * CPU oracle for the Wilson-Dirac operator -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  It shares no code with the HIP library: its
 * geometry, gamma matrices and stencil are written here from the definitions,
 * plainly and slowly, in FP64.
 *
 * Operator (the "Wilson fermion matrix" / "Wilson Dirac operator D" of the
 * paper, Sec. 1 and Sec. 4; the paper fixes no conventions, so the following
 * reading is used):
 *
 *   (D psi)(x) = psi(x) - kappa * sum_mu [ (1 - g_mu) U_mu(x)      psi(x+mu)
 *                                        + (1 + g_mu) U_mu(x-mu)^H psi(x-mu) ]
 *
 * with hermitian Euclidean gamma matrices in the chiral (DeGrand-Rossi)
 * basis, periodic boundaries, site index x + Lx*(y + Ly*(z + Lz*t)) and
 * U_mu(x) on the link x -> x+mu.  The hermitian positive definite matrix of
 * the systems (sigma_j I + A) X_j = B (Sec. 1, eqs. (1.1), (1.2)) is
 * A = D^H D.
 *
 * Array layouts (C order, complex double):
 *   U   [V][4][3][3]     U[x][mu][a][b] = (U_mu(x))_{ab}
 *   psi [V][4][3][m]     spin, colour, then right-hand side innermost
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* g[mu][row][col], mu = 0..3 for the x, y, z, t directions. */
static const cplx GAMMA[4][4][4] = {
    /* gamma_x */
    {{0, 0, 0, I}, {0, 0, I, 0}, {0, -I, 0, 0}, {-I, 0, 0, 0}},
    /* gamma_y */
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    /* gamma_z */
    {{0, 0, I, 0}, {0, 0, 0, -I}, {-I, 0, 0, 0}, {0, I, 0, 0}},
    /* gamma_t */
    {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
};

void oracle_gamma(int mu, cplx *out16)
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            out16[r * 4 + c] = GAMMA[mu][r][c];
}

static int64_t site_of(const int32_t L[4], const int c[4])
{
    return (int64_t)c[0] + (int64_t)L[0] * ((int64_t)c[1] + (int64_t)L[1] *
           ((int64_t)c[2] + (int64_t)L[2] * (int64_t)c[3]));
}

static void coords_of(const int32_t L[4], int64_t site, int c[4])
{
    for (int d = 0; d < 4; ++d) {
        c[d] = (int)(site % L[d]);
        site /= L[d];
    }
}

/* Neighbour of `site` one step in direction mu, forward (dir=+1) or
 * backward (dir=-1), with periodic wrap. */
static int64_t hop(const int32_t L[4], int64_t site, int mu, int dir)
{
    int c[4];
    coords_of(L, site, c);
    c[mu] = (c[mu] + dir + L[mu]) % L[mu];
    return site_of(L, c);
}

/* Neighbour table [V][8]: +x, -x, +y, -y, +z, -z, +t, -t. */
void oracle_neighbors(const int32_t L[4], int32_t *out)
{
    int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    for (int64_t x = 0; x < V; ++x)
        for (int mu = 0; mu < 4; ++mu) {
            out[x * 8 + 2 * mu] = (int32_t)hop(L, x, mu, +1);
            out[x * 8 + 2 * mu + 1] = (int32_t)hop(L, x, mu, -1);
        }
}

/* Apply D (dagger = 0) or D^H (dagger = 1) at one site x, writing the
 * 12*m values of the result to out[4][3][m].  in_x points at psi(x),
 * in_f[mu] at psi(x+mu) and in_b[mu] at psi(x-mu) (each a [4][3][m] block).
 *
 * D^H is written from D by taking the adjoint of each hopping term:
 * [(1 - g) U_mu(x-mu)]^H moves to the backward hop and [(1 + g) U^H]^H to the
 * forward hop, i.e. the projector signs swap. */
static void apply_D_core(const int32_t L[4], const cplx *U, double kappa, int m,
                         int dagger, int64_t x, const cplx *in_x,
                         const cplx *const in_f[4], const cplx *const in_b[4],
                         cplx *out)
{
    const double sgn = dagger ? -1.0 : 1.0;
    for (int i = 0; i < 12 * m; ++i)
        out[i] = in_x[i];

    for (int mu = 0; mu < 4; ++mu) {
        int64_t xb = hop(L, x, mu, -1);
        const cplx *Uf = U + (x * 4 + mu) * 9;   /* U_mu(x)    */
        const cplx *Ub = U + (xb * 4 + mu) * 9;  /* U_mu(x-mu) */
        const cplx *pf_in = in_f[mu];
        const cplx *pb_in = in_b[mu];
        for (int r = 0; r < m; ++r) {
            cplx chi_f[4][3], chi_b[4][3];
            /* colour multiply: chi_f = U_mu(x) psi(x+mu), chi_b = U_mu(x-mu)^H psi(x-mu) */
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a) {
                    cplx f = 0, b = 0;
                    for (int c = 0; c < 3; ++c) {
                        f += Uf[a * 3 + c] * pf_in[(s * 3 + c) * m + r];
                        b += conj(Ub[c * 3 + a]) * pb_in[(s * 3 + c) * m + r];
                    }
                    chi_f[s][a] = f;
                    chi_b[s][a] = b;
                }
            /* spin multiply with (1 - sgn g_mu) and (1 + sgn g_mu) */
            for (int al = 0; al < 4; ++al)
                for (int a = 0; a < 3; ++a) {
                    cplx acc = 0;
                    for (int be = 0; be < 4; ++be) {
                        cplx id = (al == be) ? 1.0 : 0.0;
                        cplx pf = id - sgn * GAMMA[mu][al][be];
                        cplx pb = id + sgn * GAMMA[mu][al][be];
                        acc += pf * chi_f[be][a] + pb * chi_b[be][a];
                    }
                    out[(al * 3 + a) * m + r] -= kappa * acc;
                }
        }
    }
}

/* D or D^H at site x of a full-lattice field psi[V][4][3][m]. */
static void apply_D_site(const int32_t L[4], const cplx *U, double kappa,
                         const cplx *psi, int m, int dagger, int64_t x, cplx *out)
{
    const cplx *in_f[4], *in_b[4];
    for (int mu = 0; mu < 4; ++mu) {
        in_f[mu] = psi + hop(L, x, mu, +1) * 12 * m;
        in_b[mu] = psi + hop(L, x, mu, -1) * 12 * m;
    }
    apply_D_core(L, U, kappa, m, dagger, x, psi + x * 12 * m, in_f, in_b, out);
}

/* out = D psi (dagger = 0) or D^H psi (dagger = 1) on the whole lattice. */
void oracle_apply_D(const int32_t L[4], const cplx *U, double kappa,
                    const cplx *psi, cplx *out, int32_t m, int32_t dagger)
{
    int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < V; ++x)
        apply_D_site(L, U, kappa, psi, m, dagger, x, out + x * 12 * m);
}

/* out = A psi = D^H (D psi). */
int oracle_apply_A(const int32_t L[4], const cplx *U, double kappa,
                   const cplx *psi, cplx *out, int32_t m)
{
    int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)(V * 12 * m));
    if (!tmp)
        return 1;
    oracle_apply_D(L, U, kappa, psi, tmp, m, 0);
    oracle_apply_D(L, U, kappa, tmp, out, m, 1);
    free(tmp);
    return 0;
}

/* D psi (dagger = 0) or D^H psi (dagger = 1) at the listed sites only:
 * out[k][4][3][m] holds the result at sites[k]. */
void oracle_apply_D_sites(const int32_t L[4], const cplx *U, double kappa,
                          const cplx *psi, int32_t m, int32_t dagger,
                          const int64_t *sites, int64_t nsites, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nsites; ++k)
        apply_D_site(L, U, kappa, psi, m, dagger, sites[k], out + k * 12 * m);
}

/* (A psi)(x) = (D^H (D psi))(x) at the listed sites.  D^H at x reads D psi
 * at x and at its eight neighbours, so D psi is first formed on those nine
 * sites. */
int oracle_apply_A_sites(const int32_t L[4], const cplx *U, double kappa,
                         const cplx *psi, int32_t m, const int64_t *sites,
                         int64_t nsites, cplx *out)
{
    int rc = 0;
#pragma omp parallel
    {
        cplx *Dpsi = (cplx *)malloc(sizeof(cplx) * (size_t)(9 * 12 * m));
        if (!Dpsi) {
#pragma omp atomic write
            rc = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t k = 0; k < nsites; ++k) {
                int64_t x = sites[k];
                const cplx *in_f[4], *in_b[4];
                apply_D_site(L, U, kappa, psi, m, 0, x, Dpsi);
                for (int mu = 0; mu < 4; ++mu) {
                    apply_D_site(L, U, kappa, psi, m, 0, hop(L, x, mu, +1),
                                 Dpsi + (1 + 2 * mu) * 12 * m);
                    apply_D_site(L, U, kappa, psi, m, 0, hop(L, x, mu, -1),
                                 Dpsi + (2 + 2 * mu) * 12 * m);
                    in_f[mu] = Dpsi + (1 + 2 * mu) * 12 * m;
                    in_b[mu] = Dpsi + (2 + 2 * mu) * 12 * m;
                }
                apply_D_core(L, U, kappa, m, 1, x, Dpsi, in_f, in_b, out + k * 12 * m);
            }
            free(Dpsi);
        }
    }
    return rc;
}

/*
 * Link derivative of f(U) = Re <phi, D psi> = Re sum_x phi(x)^H (D psi)(x),
 * summed over the m columns, in the convention G = df/dRe U + i df/dIm U.
 *
 * U_mu(x) enters D psi at x (forward hop) and at x+mu (backward hop through
 * U_mu(x)^H).  For f = Re c^H U d the derivative is c d^H; for
 * f = Re e^H U^H g it is g e^H.  Hence
 *
 *   G_mu(x) = -kappa sum_{spin, col} [ ((1 - g_mu) phi(x)) psi(x+mu)^H
 *                                     + psi(x) ((1 + g_mu) phi(x+mu))^H ].
 *
 * out[V][4][3][3] is overwritten.
 */
void oracle_link_grad(const int32_t L[4], double kappa, const cplx *phi,
                      const cplx *psi, int32_t m, cplx *out)
{
    int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < V; ++x) {
        for (int mu = 0; mu < 4; ++mu) {
            int64_t xf = hop(L, x, mu, +1);
            cplx G[3][3];
            memset(G, 0, sizeof(G));
            for (int r = 0; r < m; ++r) {
                for (int al = 0; al < 4; ++al) {
                    /* ((1 - g) phi(x))_al and ((1 + g) phi(x+mu))_al, per colour */
                    cplx pm[3], pp[3];
                    for (int a = 0; a < 3; ++a) {
                        cplx sm = 0, sp = 0;
                        for (int be = 0; be < 4; ++be) {
                            cplx id = (al == be) ? 1.0 : 0.0;
                            sm += (id - GAMMA[mu][al][be]) * phi[((x * 4 + be) * 3 + a) * m + r];
                            sp += (id + GAMMA[mu][al][be]) * phi[((xf * 4 + be) * 3 + a) * m + r];
                        }
                        pm[a] = sm;
                        pp[a] = sp;
                    }
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            G[a][b] += pm[a] * conj(psi[((xf * 4 + al) * 3 + b) * m + r]);
                            G[a][b] += psi[((x * 4 + al) * 3 + a) * m + r] * conj(pp[b]);
                        }
                }
            }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    out[((x * 4 + mu) * 3 + a) * 3 + b] = -kappa * G[a][b];
        }
    }
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
