// Link derivative of f(U) = sum_k Re <Phi_k, D[U] Psi_k>, the building block of
// dL/dU for the solutions X_j = (sigma_j + D^H D)^{-1} B: with
// Lambda_j = (sigma_j + A)^{-1} G_j the derivative of L is
//   -sum_j [ d Re <D Lambda_j, D X_j> + d Re <D X_j, D Lambda_j> ]
// i.e. two calls of this kernel with (Phi, Psi) = (D Lambda, X) and (D X, Lambda).
//
// U_mu(x) enters D Psi at x (forward hop) and at x+mu (backward hop through
// U_mu(x)^H).  For f = Re c^H U d the derivative dRe + i dIm is c d^H; for
// f = Re e^H U^H g it is g e^H.  Hence
//
//   G_mu(x) = -kappa sum_{spin, k} [ ((1 - g_mu) Phi(x)) Psi(x+mu)^H
//                                   + Psi(x) ((1 + g_mu) Phi(x+mu))^H ],
//
// a fused outer-product stencil: one thread per (site, mu) accumulates the
// 3 x 3 colour matrix over spins and columns in registers.

#include "grad.hpp"
#include "lattice.hpp"

namespace dsbcg {

template <int MU>
__device__ inline void grad_dir(const Geom &g, int x, const int c[4], double kappa,
                                const zd *__restrict__ Phi, const zd *__restrict__ Psi, int cols,
                                zd G[3][3]) {
    const int64_t V = g.V, n = 12 * V;
    const int xf = hop(g, x, c, MU, true);
    for (int k = 0; k < cols; ++k) {
        const zd *ph = Phi + (int64_t)k * n;
        const zd *ps = Psi + (int64_t)k * n;
        zd p[4][3], a[4][3];
        // ((1 - g_mu) Phi(x)) Psi(x+mu)^H
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int q = 0; q < 3; ++q) p[s][q] = ph[(int64_t)(s * 3 + q) * V + x];
        project_full<double, MU, 1>(p, a);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            zd y[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) y[q] = ps[(int64_t)(s * 3 + q) * V + xf];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) cmac_conj(G[i][j], y[j], a[s][i]);
        }
        // Psi(x) ((1 + g_mu) Phi(x+mu))^H
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int q = 0; q < 3; ++q) p[s][q] = ph[(int64_t)(s * 3 + q) * V + xf];
        project_full<double, MU, -1>(p, a);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            zd y[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) y[q] = ps[(int64_t)(s * 3 + q) * V + x];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) cmac_conj(G[i][j], a[s][j], y[i]);
        }
    }
}

__global__ __launch_bounds__(256) void link_grad_kernel(Geom g, double kappa, const zd *__restrict__ Phi,
                                                        const zd *__restrict__ Psi, int cols,
                                                        zd *__restrict__ dU, int accumulate,
                                                        double scale) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 4 * (int64_t)g.V) return;
    const int mu = (int)(t / g.V);
    const int x = (int)(t - (int64_t)mu * g.V);
    int c[4];
    site_coords(g, x, c);
    zd G[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) G[i][j] = mk<double>(0, 0);
    if (mu == 0) grad_dir<0>(g, x, c, kappa, Phi, Psi, cols, G);
    else if (mu == 1) grad_dir<1>(g, x, c, kappa, Phi, Psi, cols, G);
    else if (mu == 2) grad_dir<2>(g, x, c, kappa, Phi, Psi, cols, G);
    else grad_dir<3>(g, x, c, kappa, Phi, Psi, cols, G);
    zd *o = dU + ((int64_t)x * 4 + mu) * 9;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const zd v = mk<double>(-scale * kappa * G[i][j].x, -scale * kappa * G[i][j].y);
            o[i * 3 + j] = accumulate ? o[i * 3 + j] + v : v;
        }
}

hipError_t link_grad_apply(const Geom &g, double kappa, const void *Phi, const void *Psi, int cols,
                           void *dU, bool accumulate, double scale, hipStream_t st) {
    const int64_t total = 4 * (int64_t)g.V;
    hipLaunchKernelGGL(link_grad_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g,
                       kappa, (const zd *)Phi, (const zd *)Psi, cols, (zd *)dU, accumulate ? 1 : 0, scale);
    return hipGetLastError();
}

}  // namespace dsbcg
