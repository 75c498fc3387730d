// Wilson-Dirac stencil D and D^H on a block of right-hand sides (gfx950).
//
//   (D psi)(x) = psi(x) - kappa sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
//                                      + (1 + g_mu) U_mu(x-mu)^H psi(x-mu) ]
//
// and D^H with the projector signs swapped.  This is the "Wilson fermion
// matrix" of Sec. 1 of the paper (A = D^H D is the hpd matrix of eq. (1.1));
// the paper stores it as a general sparse matrix (Sec. 4), here it is a
// matrix-free stencil.
//
// One thread computes the 12 spin-colour components of one (site, column)
// pair.  Each hop first projects the neighbour spinor onto the two-spin
// subspace of (1 -+ g_mu) (6 complex numbers), multiplies those by the SU(3)
// link and rebuilds the four spin components from them.  The link matrices
// of a workgroup's sites are staged once in LDS and shared by the NB columns
// of each site.
//
// Gamma matrices (chiral basis):
//   g_x = [[0,0,0,i],[0,0,i,0],[0,-i,0,0],[-i,0,0,0]]
//   g_y = [[0,0,0,-1],[0,0,1,0],[0,1,0,0],[-1,0,0,0]]
//   g_z = [[0,0,i,0],[0,0,0,-i],[-i,0,0,0],[0,i,0,0]]
//   g_t = [[0,0,1,0],[0,0,0,1],[1,0,0,0],[0,1,0,0]]
// For P = 1 - s g_mu (s = +-1) the image is fixed by spins 0 and 1:
//   x: h0 = p0 - s i p3, h1 = p1 - s i p2;  P p = [h0, h1,  s i h1,  s i h0]
//   y: h0 = p0 + s p3,   h1 = p1 - s p2;    P p = [h0, h1, -s h1,    s h0]
//   z: h0 = p0 - s i p2, h1 = p1 + s i p3;  P p = [h0, h1,  s i h0, -s i h1]
//   t: h0 = p0 - s p2,   h1 = p1 - s p3;    P p = [h0, h1, -s h0,   -s h1]
// and P commutes with the colour multiply, so U (P p) = P (U p) is formed
// from U h0 and U h1.

#include "stencil.hpp"

namespace dsbcg {

__device__ inline void site_coords(const Geom &g, int x, int c[4]) {
    c[0] = x % g.L[0];
    x /= g.L[0];
    c[1] = x % g.L[1];
    x /= g.L[1];
    c[2] = x % g.L[2];
    c[3] = x / g.L[2];
}

// Neighbour of site x (coordinates c) one step along mu, forward or backward.
__device__ inline int hop(const Geom &g, int x, const int c[4], int mu, bool fwd) {
    int stride = 1;
    for (int d = 0; d < mu; ++d) stride *= g.L[d];
    if (fwd) return (c[mu] == g.L[mu] - 1) ? x - (g.L[mu] - 1) * stride : x + stride;
    return (c[mu] == 0) ? x + (g.L[mu] - 1) * stride : x - stride;
}

template <typename R, int MU, int S>
__device__ inline void project(const cx<R> p[4][3], cx<R> h[2][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (MU == 0) {
            h[0][a] = (S > 0) ? p[0][a] - mul_i(p[3][a]) : p[0][a] + mul_i(p[3][a]);
            h[1][a] = (S > 0) ? p[1][a] - mul_i(p[2][a]) : p[1][a] + mul_i(p[2][a]);
        } else if (MU == 1) {
            h[0][a] = (S > 0) ? p[0][a] + p[3][a] : p[0][a] - p[3][a];
            h[1][a] = (S > 0) ? p[1][a] - p[2][a] : p[1][a] + p[2][a];
        } else if (MU == 2) {
            h[0][a] = (S > 0) ? p[0][a] - mul_i(p[2][a]) : p[0][a] + mul_i(p[2][a]);
            h[1][a] = (S > 0) ? p[1][a] + mul_i(p[3][a]) : p[1][a] - mul_i(p[3][a]);
        } else {
            h[0][a] = (S > 0) ? p[0][a] - p[2][a] : p[0][a] + p[2][a];
            h[1][a] = (S > 0) ? p[1][a] - p[3][a] : p[1][a] + p[3][a];
        }
    }
}

template <typename R, int MU, int S>
__device__ inline void reconstruct_add(cx<R> acc[4][3], const cx<R> u[2][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[0][a] = acc[0][a] + u[0][a];
        acc[1][a] = acc[1][a] + u[1][a];
        if (MU == 0) {
            acc[2][a] = (S > 0) ? acc[2][a] + mul_i(u[1][a]) : acc[2][a] - mul_i(u[1][a]);
            acc[3][a] = (S > 0) ? acc[3][a] + mul_i(u[0][a]) : acc[3][a] - mul_i(u[0][a]);
        } else if (MU == 1) {
            acc[2][a] = (S > 0) ? acc[2][a] - u[1][a] : acc[2][a] + u[1][a];
            acc[3][a] = (S > 0) ? acc[3][a] + u[0][a] : acc[3][a] - u[0][a];
        } else if (MU == 2) {
            acc[2][a] = (S > 0) ? acc[2][a] + mul_i(u[0][a]) : acc[2][a] - mul_i(u[0][a]);
            acc[3][a] = (S > 0) ? acc[3][a] - mul_i(u[1][a]) : acc[3][a] + mul_i(u[1][a]);
        } else {
            acc[2][a] = (S > 0) ? acc[2][a] - u[0][a] : acc[2][a] + u[0][a];
            acc[3][a] = (S > 0) ? acc[3][a] - u[1][a] : acc[3][a] + u[1][a];
        }
    }
}

template <typename R>
__device__ inline void load_spinor(const cx<R> *__restrict__ in, int64_t base, int64_t comp,
                                   cx<R> p[4][3]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) p[s][a] = in[base + (s * 3 + a) * comp];
}

// One hop in direction MU with projector sign S: acc += P (W h) where W is
// the link (ADJ = false) or its adjoint (ADJ = true).
template <typename R, int MU, int S, bool ADJ>
__device__ inline void hop_term(cx<R> acc[4][3], const cx<R> *__restrict__ lnk,
                                const cx<R> p[4][3]) {
    cx<R> h[2][3], u[2][3];
    project<R, MU, S>(p, h);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<R> t = mk<R>(0, 0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (ADJ)
                    cmac_conj(t, lnk[b * 3 + a], h[k][b]);
                else
                    cmac(t, lnk[a * 3 + b], h[k][b]);
            }
            u[k][a] = t;
        }
    reconstruct_add<R, MU, S>(acc, u);
}

template <typename R, int MU, bool DAG, bool LDS>
__device__ inline void direction(cx<R> acc[4][3], const Geom &g, int x, const int c[4],
                                 const cx<R> *__restrict__ U, const cx<R> *lf, const cx<R> *lb,
                                 const cx<R> *__restrict__ in, int64_t in_site, int64_t in_comp,
                                 int r) {
    constexpr int SF = DAG ? -1 : 1;  // forward hop uses 1 - SF g_mu
    cx<R> p[4][3];
    const int xf = hop(g, x, c, MU, true);
    load_spinor(in, (int64_t)xf * in_site + r, in_comp, p);
    hop_term<R, MU, SF, false>(acc, LDS ? lf + MU * 9 : U + ((int64_t)x * 4 + MU) * 9, p);
    const int xb = hop(g, x, c, MU, false);
    load_spinor(in, (int64_t)xb * in_site + r, in_comp, p);
    hop_term<R, MU, -SF, true>(acc, LDS ? lb + MU * 9 : U + ((int64_t)xb * 4 + MU) * 9, p);
}

template <typename R, int NB, bool LDS>
struct StencilShape {
    // sites per workgroup; with LDS staging the links of a site take
    // 72 complex numbers, so the site count is capped to keep a workgroup's
    // LDS near 55 KB.
    static constexpr int cap = LDS ? (sizeof(R) == 8 ? 48 : 96) : 256;
    static constexpr int want = (256 / NB) > 0 ? 256 / NB : 1;
    static constexpr int SPW = want < cap ? want : cap;
    static constexpr int THREADS = SPW * NB;
};

template <typename R, int NB, bool DAG, bool LDS>
__global__ __launch_bounds__((StencilShape<R, NB, LDS>::THREADS)) void wilson_kernel(
    Geom g, const cx<R> *__restrict__ U, R kappa, const cx<R> *__restrict__ in,
    int64_t in_site, int64_t in_comp, cx<R> *__restrict__ out, int64_t out_site,
    int64_t out_comp) {
    using SH = StencilShape<R, NB, LDS>;
    constexpr int SPW = SH::SPW;
    __shared__ cx<R> lds_links[LDS ? 2 * SPW * 36 : 1];
    cx<R> *lf = lds_links;
    cx<R> *lb = lds_links + (LDS ? SPW * 36 : 0);

    const int s0 = blockIdx.x * SPW;
    const int nsites = min(SPW, g.V - s0);
    if (LDS) {
        // forward links U_mu(x) of this workgroup's sites: one contiguous chunk
        for (int k = threadIdx.x; k < nsites * 36; k += SH::THREADS)
            lf[k] = U[(int64_t)s0 * 36 + k];
        // backward links U_mu(x - mu)
        for (int k = threadIdx.x; k < nsites * 36; k += SH::THREADS) {
            const int sl = k / 36, rem = k - sl * 36, mu = rem / 9, e = rem - mu * 9;
            int c[4];
            const int x = s0 + sl;
            site_coords(g, x, c);
            const int xb = hop(g, x, c, mu, false);
            lb[k] = U[((int64_t)xb * 4 + mu) * 9 + e];
        }
        __syncthreads();
    }

    const int sl = threadIdx.x / NB;
    const int r = threadIdx.x - sl * NB;
    if (sl >= nsites) return;
    const int x = s0 + sl;
    int c[4];
    site_coords(g, x, c);

    cx<R> acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[s][a] = mk<R>(0, 0);

    const cx<R> *lfs = lf + sl * 36;
    const cx<R> *lbs = lb + sl * 36;
    direction<R, 0, DAG, LDS>(acc, g, x, c, U, lfs, lbs, in, in_site, in_comp, r);
    direction<R, 1, DAG, LDS>(acc, g, x, c, U, lfs, lbs, in, in_site, in_comp, r);
    direction<R, 2, DAG, LDS>(acc, g, x, c, U, lfs, lbs, in, in_site, in_comp, r);
    direction<R, 3, DAG, LDS>(acc, g, x, c, U, lfs, lbs, in, in_site, in_comp, r);

    const int64_t ib = (int64_t)x * in_site + r;
    const int64_t ob = (int64_t)x * out_site + r;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const cx<R> v = in[ib + (s * 3 + a) * in_comp];
            out[ob + (s * 3 + a) * out_comp] = mk<R>(v.x - kappa * acc[s][a].x,
                                                     v.y - kappa * acc[s][a].y);
        }
}

__global__ void neighbor_kernel(Geom g, int32_t *out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.V) return;
    int c[4];
    site_coords(g, x, c);
    for (int mu = 0; mu < 4; ++mu) {
        out[(int64_t)x * 8 + 2 * mu] = hop(g, x, c, mu, true);
        out[(int64_t)x * 8 + 2 * mu + 1] = hop(g, x, c, mu, false);
    }
}

template <typename R, int NB, bool LDS>
static hipError_t launch_nb(const Geom &g, const void *U, double kappa, const void *in,
                            int64_t in_site, int64_t in_comp, void *out, int64_t out_site,
                            int64_t out_comp, bool dagger, hipStream_t st) {
    using SH = StencilShape<R, NB, LDS>;
    const dim3 grid((g.V + SH::SPW - 1) / SH::SPW);
    const dim3 block(SH::THREADS);
    if (dagger)
        hipLaunchKernelGGL((wilson_kernel<R, NB, true, LDS>), grid, block, 0, st, g,
                           (const cx<R> *)U, (R)kappa, (const cx<R> *)in, in_site, in_comp,
                           (cx<R> *)out, out_site, out_comp);
    else
        hipLaunchKernelGGL((wilson_kernel<R, NB, false, LDS>), grid, block, 0, st, g,
                           (const cx<R> *)U, (R)kappa, (const cx<R> *)in, in_site, in_comp,
                           (cx<R> *)out, out_site, out_comp);
    return hipGetLastError();
}

template <typename R, bool LDS>
static hipError_t launch_prec(const Geom &g, const void *U, double kappa, const void *in,
                              int64_t in_site, int64_t in_comp, void *out, int64_t out_site,
                              int64_t out_comp, int nb, bool dagger, hipStream_t st) {
    switch (nb) {
#define DSBCG_NB_CASE(N)                                                                  \
    case N:                                                                               \
        return launch_nb<R, N, LDS>(g, U, kappa, in, in_site, in_comp, out, out_site,     \
                                    out_comp, dagger, st);
        DSBCG_NB_CASE(1) DSBCG_NB_CASE(2) DSBCG_NB_CASE(3) DSBCG_NB_CASE(4)
        DSBCG_NB_CASE(5) DSBCG_NB_CASE(6) DSBCG_NB_CASE(7) DSBCG_NB_CASE(8)
        DSBCG_NB_CASE(9) DSBCG_NB_CASE(10) DSBCG_NB_CASE(11) DSBCG_NB_CASE(12)
        DSBCG_NB_CASE(13) DSBCG_NB_CASE(14) DSBCG_NB_CASE(15) DSBCG_NB_CASE(16)
#undef DSBCG_NB_CASE
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t wilson_apply(const Geom &g, bool fp64, const void *U, double kappa, const void *in,
                        int64_t in_site, int64_t in_comp, void *out, int64_t out_site,
                        int64_t out_comp, int nb, bool dagger, bool lds_links, hipStream_t st) {
    if (fp64)
        return lds_links ? launch_prec<double, true>(g, U, kappa, in, in_site, in_comp, out,
                                                     out_site, out_comp, nb, dagger, st)
                         : launch_prec<double, false>(g, U, kappa, in, in_site, in_comp, out,
                                                      out_site, out_comp, nb, dagger, st);
    return lds_links ? launch_prec<float, true>(g, U, kappa, in, in_site, in_comp, out,
                                                out_site, out_comp, nb, dagger, st)
                     : launch_prec<float, false>(g, U, kappa, in, in_site, in_comp, out,
                                                 out_site, out_comp, nb, dagger, st);
}

hipError_t neighbor_table(const Geom &g, int32_t *dev_out, hipStream_t st) {
    hipLaunchKernelGGL(neighbor_kernel, dim3((g.V + 255) / 256), dim3(256), 0, st, g, dev_out);
    return hipGetLastError();
}

}  // namespace dsbcg
