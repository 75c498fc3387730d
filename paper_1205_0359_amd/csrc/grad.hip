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
// a fused outer-product stencil.  (1 - s g_mu) is hermitian and its image
// is fixed by the half spinor h(p) = (h_0, h_1) of spins 0 and 1, with the
// lower spins unit multiples of them, so the spin sums reduce to half spinors:
//   sum_spin ((1 - s g_mu) p) y^H = sum_{k=0,1} h_k(p) h_k(y)^H
// (same mu and s on both sides).  One thread per (site, mu), mu the fastest
// index: the four threads of a site are neighbouring lanes, read Phi(x) and
// Psi(x) together and write the site's four 3 x 3 blocks as one contiguous
// run.

#include "grad.hpp"
#include "lattice.hpp"

namespace dsbcg {

// Half spinor of the projector (1 - s g_mu) with mu a runtime value (no
// divergence between the lanes of different mu): h_k = p_k + f_k p_partner,
// partner 3 - k for x, y and 2 + k for z, t, f_k = s * (x: -i, -i;
// y: +1, -1; z: -i, +i; t: -1, -1).  Loads the 12 components of the spinor
// at site x of the column-major field f.
__device__ inline void half_rt(int mu, double sgn, const zd *__restrict__ f, int64_t V, int x,
                               zd h[2][3]) {
    const bool xy = mu < 2;
    const double fr[2] = {sgn * (mu == 1 ? 1.0 : (mu == 3 ? -1.0 : 0.0)),
                          sgn * (mu == 1 ? -1.0 : (mu == 3 ? -1.0 : 0.0))};
    const double fi[2] = {sgn * ((mu == 0 || mu == 2) ? -1.0 : 0.0),
                          sgn * (mu == 0 ? -1.0 : (mu == 2 ? 1.0 : 0.0))};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int partner = xy ? 3 - k : 2 + k;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const zd a = f[(int64_t)(k * 3 + q) * V + x];
            const zd b = f[(int64_t)(partner * 3 + q) * V + x];
            h[k][q] = mk<double>(a.x + fr[k] * b.x - fi[k] * b.y, a.y + fr[k] * b.y + fi[k] * b.x);
        }
    }
}

__global__ __launch_bounds__(256) void link_grad_kernel(Geom g, double kappa, const zd *__restrict__ Phi,
                                                        const zd *__restrict__ Psi, int cols,
                                                        zd *__restrict__ dU, int accumulate,
                                                        double scale) {
    // the workgroup's 64 sites x 4 directions x 9 entries, written out as one
    // contiguous run after the barrier
    __shared__ zd out[256 * 9];
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t total = 4 * (int64_t)g.V;
    zd G[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) G[i][j] = mk<double>(0, 0);
    if (t < total) {
        const int mu = (int)(t & 3);
        const int x = (int)(t >> 2);
        const int64_t V = g.V, n = 12 * V;
        int c[4];
        site_coords(g, x, c);
        const int s1 = g.L[0], s2 = s1 * g.L[1], s3 = s2 * g.L[2];
        const int stride = mu == 0 ? 1 : (mu == 1 ? s1 : (mu == 2 ? s2 : s3));
        const int cm = mu == 0 ? c[0] : (mu == 1 ? c[1] : (mu == 2 ? c[2] : c[3]));
        const int lm = g.L[mu];
        const int xf = x + stride - (cm == lm - 1 ? lm * stride : 0);
        for (int k = 0; k < cols; ++k) {
            const zd *ph = Phi + (int64_t)k * n;
            const zd *ps = Psi + (int64_t)k * n;
            zd a[2][3], b[2][3];
            // ((1 - g_mu) Phi(x)) Psi(x+mu)^H
            half_rt(mu, 1.0, ph, V, x, a);
            half_rt(mu, 1.0, ps, V, xf, b);
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) cmac_conj(G[i][j], b[h][j], a[h][i]);
            // Psi(x) ((1 + g_mu) Phi(x+mu))^H
            half_rt(mu, -1.0, ps, V, x, a);
            half_rt(mu, -1.0, ph, V, xf, b);
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) cmac_conj(G[i][j], b[h][j], a[h][i]);
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            out[threadIdx.x * 9 + i * 3 + j] = mk<double>(-scale * kappa * G[i][j].x, -scale * kappa * G[i][j].y);
    __syncthreads();
    // dU[x][mu][3][3] with t = 4 x + mu: the block's entries are contiguous
    zd *o = dU + (int64_t)blockIdx.x * blockDim.x * 9;
    const int64_t left = 9 * (total - (int64_t)blockIdx.x * blockDim.x);
    const int cnt = (int)(left < 9 * (int64_t)blockDim.x ? left : 9 * (int64_t)blockDim.x);
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) o[e] = accumulate ? o[e] + out[e] : out[e];
}

hipError_t link_grad_apply(const Geom &g, double kappa, const void *Phi, const void *Psi, int cols,
                           void *dU, bool accumulate, double scale, hipStream_t st) {
    const int64_t total = 4 * (int64_t)g.V;
    hipLaunchKernelGGL(link_grad_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g,
                       kappa, (const zd *)Phi, (const zd *)Psi, cols, (zd *)dU, accumulate ? 1 : 0, scale);
    return hipGetLastError();
}

}  // namespace dsbcg
