// Lattice geometry and spin-projection helpers shared by the stencil kernels.
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
#pragma once

#include "common.hpp"
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

// Neighbour of site x (coordinates c) one step along mu, forward or backward
// (periodic).  Written with selects rather than branches so that the hops of
// a stencil stay straight-line code.
__device__ inline int hop(const Geom &g, int x, const int c[4], int mu, bool fwd) {
    int stride = 1;
    for (int d = 0; d < mu; ++d) stride *= g.L[d];
    const int wrap = g.L[mu] * stride;
    return fwd ? x + stride - (c[mu] == g.L[mu] - 1 ? wrap : 0)
               : x - stride + (c[mu] == 0 ? wrap : 0);
}

// Spin indices (a, b) that form the half spinor h_k = p_a + coef * p_b for
// direction MU and projector sign S, and the rebuild of the lower spins.
template <int MU, int S, int K>
struct Half {
    // first spin of h_K is K; partner spin:
    static constexpr int partner = (MU == 0 || MU == 1) ? 3 - K : 2 + K;
};

// h = p_K + f * p_partner, with f one of {+1, -1, +i, -i} fixed by MU, S, K.
template <typename R, int MU, int S, int K>
__device__ inline cx<R> half(cx<R> pa, cx<R> pb) {
    if (MU == 0) return (S > 0) ? pa - mul_i(pb) : pa + mul_i(pb);               // -s i
    if (MU == 1) return (K == 0) == (S > 0) ? pa + pb : pa - pb;                   // +s, -s
    if (MU == 2) return (K == 0) == (S > 0) ? pa - mul_i(pb) : pa + mul_i(pb);     // -s i, +s i
    return (S > 0) ? pa - pb : pa + pb;                                           // -s
}

// acc (spins K and partner) += rebuild of u = W h_K.
template <typename R, int MU, int S, int K>
__device__ inline void rebuild_add(cx<R> acc[4][3], const cx<R> u[3]) {
    constexpr int P = Half<MU, S, K>::partner;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[K][a] = acc[K][a] + u[a];
        if (MU == 0) acc[P][a] = (S > 0) ? acc[P][a] + mul_i(u[a]) : acc[P][a] - mul_i(u[a]);
        if (MU == 1) acc[P][a] = ((K == 0) == (S > 0)) ? acc[P][a] + u[a] : acc[P][a] - u[a];
        if (MU == 2) acc[P][a] = ((K == 0) == (S > 0)) ? acc[P][a] + mul_i(u[a]) : acc[P][a] - mul_i(u[a]);
        if (MU == 3) acc[P][a] = (S > 0) ? acc[P][a] - u[a] : acc[P][a] + u[a];
    }
}


// a = (1 - S g_mu) p on a full spinor.
template <typename R, int MU, int S>
__device__ inline void project_full(const cx<R> p[4][3], cx<R> a[4][3]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) a[s][c] = mk<R>(0, 0);
    cx<R> h[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) h[c] = half<R, MU, S, 0>(p[0][c], p[Half<MU, S, 0>::partner][c]);
    rebuild_add<R, MU, S, 0>(a, h);
#pragma unroll
    for (int c = 0; c < 3; ++c) h[c] = half<R, MU, S, 1>(p[1][c], p[Half<MU, S, 1>::partner][c]);
    rebuild_add<R, MU, S, 1>(a, h);
}

}  // namespace dsbcg
