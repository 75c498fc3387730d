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
// Data layout: a block of nb columns is column-major over sites, element
// (column r, spin-colour c, site x) at (r*12 + c)*V + x; the links are
// structure-of-arrays, element e of U_mu(x) at (mu*9 + e)*V + x.  A workgroup
// owns 64 consecutive sites and has one wave per column, so every lane of a
// wave reads consecutive addresses.  Per direction the 64 forward links
// U_mu(x) and backward links U_mu(x-mu) of the workgroup are staged once in
// LDS and shared by all nb columns; the FP64 kernel for 5 to 7 columns
// instead lets every wave read the links from global memory (the nb waves
// read the same addresses, so the copies after the first come from cache)
// and runs without barriers.
//
// Each hop first projects the neighbour spinor onto the two-spin subspace of
// (1 -+ g_mu) (6 complex numbers), multiplies those by the SU(3) link and
// rebuilds the four spin components from them.
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

#include "lattice.hpp"
#include "stencil.hpp"

namespace dsbcg {

constexpr int kSitesPerWG = 64;

// One hop: acc += P_s (W psi(y)) with W = link (ADJ false) or link^H.
// psi is read at site y of column base `col`; element e = 0..8 of the link
// matrix is lnk[e * ls] (ls = 64 for the LDS tile, V for the global copy).
template <typename R, int MU, int S, bool ADJ>
__device__ inline void hop_term(cx<R> acc[4][3], const cx<R> *lnk, int64_t ls, const cx<R> *__restrict__ col,
                                int64_t V, int y) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int Pt = (MU == 0 || MU == 1) ? 3 - k : 2 + k;  // partner spin of h_k
        cx<R> h[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const cx<R> pa = col[(int64_t)(k * 3 + a) * V + y];
            const cx<R> pb = col[(int64_t)(Pt * 3 + a) * V + y];
            h[a] = (k == 0) ? half<R, MU, S, 0>(pa, pb) : half<R, MU, S, 1>(pa, pb);
        }
        cx<R> u[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<R> t = mk<R>(0, 0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (ADJ)
                    cmac_conj(t, lnk[(b * 3 + a) * ls], h[b]);
                else
                    cmac(t, lnk[(a * 3 + b) * ls], h[b]);
            }
            u[a] = t;
        }
        if (k == 0)
            rebuild_add<R, MU, S, 0>(acc, u);
        else
            rebuild_add<R, MU, S, 1>(acc, u);
    }
}

// Stage U_mu(x) and U_mu(x - mu) of the workgroup's sites in LDS.
template <typename R>
__device__ inline void stage_links(cx<R> *lf, cx<R> *lb, const cx<R> *__restrict__ Ul, int64_t V,
                                   int mu, int x, int xb, bool valid, int lane, int wave, int nwaves) {
    for (int e = wave; e < 9; e += nwaves) {
        if (valid) {
            lf[e * kSitesPerWG + lane] = Ul[(int64_t)(mu * 9 + e) * V + x];
            lb[e * kSitesPerWG + lane] = Ul[(int64_t)(mu * 9 + e) * V + xb];
        }
    }
}

template <typename R, int MU, bool DAG>
__device__ inline void direction(cx<R> acc[4][3], const Geom &g, int x, const int c[4],
                                 const cx<R> *__restrict__ Ul, cx<R> *lf, cx<R> *lb,
                                 const cx<R> *__restrict__ col, bool valid, int lane, int wave,
                                 int nwaves) {
    constexpr int SF = DAG ? -1 : 1;  // forward hop uses 1 - SF g_mu
    const int xf = valid ? hop(g, x, c, MU, true) : 0;
    const int xb = valid ? hop(g, x, c, MU, false) : 0;
    __syncthreads();  // previous direction finished with the LDS links
    stage_links<R>(lf, lb, Ul, g.V, MU, x, xb, valid, lane, wave, nwaves);
    __syncthreads();
    if (!valid) return;
    hop_term<R, MU, SF, false>(acc, lf + lane, kSitesPerWG, col, g.V, xf);
    hop_term<R, MU, -SF, true>(acc, lb + lane, kSitesPerWG, col, g.V, xb);
}

// The same hops with the links read from the structure-of-arrays copy in
// global memory (no LDS, no barrier).
template <typename R, int MU, bool DAG>
__device__ inline void direction_global(cx<R> acc[4][3], const Geom &g, int x, const int c[4],
                                        const cx<R> *__restrict__ Ul, const cx<R> *__restrict__ col) {
    constexpr int SF = DAG ? -1 : 1;
    const int xf = hop(g, x, c, MU, true);
    const int xb = hop(g, x, c, MU, false);
    const cx<R> *u = Ul + (int64_t)MU * 9 * g.V;
    hop_term<R, MU, SF, false>(acc, u + x, g.V, col, g.V, xf);
    hop_term<R, MU, -SF, true>(acc, u + xb, g.V, col, g.V, xb);
}

// RESID: instead of storing y = D^H in (in = D x), accumulate the squared
// norm of b - sigma x - y per column: wave w (column w) of workgroup q
// writes its sum to partials[w * (workgroups) + q].  One pass then yields the true residual
// norms ||b - (sigma + A) x|| without writing A x.
struct ResidOut {
    const zd *b;       // column-major, like in
    const zd *x;
    double sigma;
    double *partials;  // [workgroups][16]
};

// MAXT: the largest block the instantiation is launched with (64 threads per
// column).  A 512-thread bound lets the FP64 kernel keep its 138 registers
// without spills, at 3 waves per SIMD instead of 4 (1024-thread bound: 128
// registers and spills).  GL: links read from global memory by every wave
// instead of staged in LDS behind two barriers per direction (FP64: 144
// registers, 3 waves per SIMD).  Measured on 32^3 x 64 (FP64, D pass): with
// 5, 6 and 7 columns the GL form takes 2.13, 2.82 and 3.17 ms against 2.43,
// 3.05 and 3.62 ms; with 4 and 8 columns the LDS form is as fast or faster,
// and so it is for FP32 at every width measured (2 to 12).
inline bool small_bound(int nb) { return nb <= 8; }
inline bool global_links(bool fp64, int nb) { return fp64 && nb >= 5 && nb <= 7; }

// The FP64 pass costs 425 us per column at 5 columns (GL form) but 478-511 us
// per column in one launch of 8-16 columns (32^3 x 64).  Launches of 5, then
// one of 3-7 columns, were measured 6 % (8 columns), 9 % (12) and 16 % (16)
// faster than one launch, with bitwise equal results.  FP32 costs about the
// same per column at every width and is not split.
int stencil_chunk(bool fp64, int nb) { return (fp64 && nb > 7) ? 5 : nb; }

// Block order.  Workgroups are dealt to the 8 XCDs of the chip round robin
// (workgroup q runs on XCD q mod 8), and each XCD has its own L2.  In the
// plain order workgroup q owns sites 64 q .. 64 q + 63, so the y neighbours
// one workgroup over sit in another XCD's cache.  The lockstep order used by
// every launch gives XCD k the tiles k tpx .. (k+1) tpx - 1 of 64 sites of
// every t-slice and walks t: the workgroups an XCD runs at one time cover a
// block of neighbouring tiles of one slice, and their x, y, z neighbours
// mostly sit in the same L2.  The output goes out with non-temporal stores,
// which keep it from displacing the inputs in L2.  Measured on 32^3 x 64
// against the plain order, bitwise equal results: FP64 with global links,
// 5 columns, 2.02 against 2.16 ms per pass (L2-to-fabric reads 11.7 GB
// against 12.6 GB; the algorithmic reads are 3.2 GB); LDS-staged forms 2 to
// 13 % faster (FP64 3 and 4 columns 1.30 / 1.62 against 1.49 / 1.84 ms, FP32
// 5 and 12 columns 1.13 / 2.74 against 1.16 / 2.96 ms).  Walking an XCD's
// share of a slice in smaller chunks over all t (so that the t neighbours
// were read fewer workgroups earlier) was slower: 2.18, 2.36 and 2.46 ms for
// chunks of 32, 16 and 8 tiles against 2.02 ms for the whole share of 64.
struct BlockOrder {
    int32_t vs;     // sites per t-slice, Lx Ly Lz
    int32_t ntile;  // tiles of 64 sites per slice
    int32_t tpx;    // tiles per XCD
};
constexpr int kXcds = 8;
inline BlockOrder lockstep_order(const Geom &g) {
    BlockOrder o;
    o.vs = g.L[0] * g.L[1] * g.L[2];
    o.ntile = (o.vs + kSitesPerWG - 1) / kSitesPerWG;
    o.tpx = (o.ntile + kXcds - 1) / kXcds;
    return o;
}
inline int lockstep_blocks(const Geom &g) { return kXcds * lockstep_order(g).tpx * g.L[3]; }

template <typename R, bool DAG, bool RESID, int MAXT, bool GL>
__global__ __launch_bounds__(MAXT) void wilson_cm_kernel(Geom g, const cx<R> *__restrict__ Ul,
                                                         R kappa, const cx<R> *__restrict__ in,
                                                         cx<R> *__restrict__ out, int nb, ResidOut ro,
                                                         BlockOrder bo, ApiOut ao) {
    __shared__ cx<R> lf[9 * kSitesPerWG];
    __shared__ cx<R> lb[9 * kSitesPerWG];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;  // = column
    const int nwaves = blockDim.x >> 6;
    // lockstep block order
    const int xcd = blockIdx.x % kXcds, q = blockIdx.x / kXcds;
    const int t = q / bo.tpx, tile = xcd * bo.tpx + (q - t * bo.tpx);
    const int xs = tile * kSitesPerWG + lane;
    const bool inside = tile < bo.ntile && t < g.L[3] && xs < bo.vs;
    const int x = t * bo.vs + xs;
    const bool valid = inside && wave < nb;
    int c[4] = {0, 0, 0, 0};
    if (valid) site_coords(g, x, c);
    const int64_t n = 12 * (int64_t)g.V;
    const cx<R> *col = in + (int64_t)wave * n;

    cx<R> acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[s][a] = mk<R>(0, 0);

    if (GL) {
        if (valid) {
            direction_global<R, 0, DAG>(acc, g, x, c, Ul, col);
            direction_global<R, 1, DAG>(acc, g, x, c, Ul, col);
            direction_global<R, 2, DAG>(acc, g, x, c, Ul, col);
            direction_global<R, 3, DAG>(acc, g, x, c, Ul, col);
        }
    } else {
        direction<R, 0, DAG>(acc, g, x, c, Ul, lf, lb, col, valid, lane, wave, nwaves);
        direction<R, 1, DAG>(acc, g, x, c, Ul, lf, lb, col, valid, lane, wave, nwaves);
        direction<R, 2, DAG>(acc, g, x, c, Ul, lf, lb, col, valid, lane, wave, nwaves);
        direction<R, 3, DAG>(acc, g, x, c, Ul, lf, lb, col, valid, lane, wave, nwaves);
    }
    if (RESID) {
        double r2 = 0.0;
        if (valid) {
            const int64_t base = (int64_t)wave * n;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int64_t idx = (int64_t)(s * 3 + a) * g.V + x;
                    const cx<R> v = col[idx];
                    const double yr = (double)v.x - (double)kappa * (double)acc[s][a].x;
                    const double yi = (double)v.y - (double)kappa * (double)acc[s][a].y;
                    const zd bv = ro.b[base + idx], xv = ro.x[base + idx];
                    const double rr = bv.x - ro.sigma * xv.x - yr, ri = bv.y - ro.sigma * xv.y - yi;
                    r2 += rr * rr + ri * ri;
                }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) r2 += __shfl_xor(r2, off, 64);
        if (lane == 0 && wave < nb) ro.partials[(int64_t)wave * gridDim.x + blockIdx.x] = r2;
        return;
    }
    if (!valid) return;

    if (ao.y) {
        // the caller's layout: the 12 components of a site and its m
        // columns are one contiguous run, which the nb waves of the
        // workgroup fill together in L2 (plain stores)
        zd *oy = (zd *)ao.y + (int64_t)x * 12 * ao.m + ao.c0 + wave;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const cx<R> v = col[(int64_t)(s * 3 + a) * g.V + x];
                const cx<R> r = mk<R>(v.x - kappa * acc[s][a].x, v.y - kappa * acc[s][a].y);
                oy[(s * 3 + a) * ao.m] = mk<double>((double)r.x, (double)r.y);
            }
        return;
    }
    cx<R> *oc = out + (int64_t)wave * n;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int64_t idx = (int64_t)(s * 3 + a) * g.V + x;
            const cx<R> v = col[idx];
            const cx<R> r = mk<R>(v.x - kappa * acc[s][a].x, v.y - kappa * acc[s][a].y);
            __builtin_nontemporal_store(r.x, &oc[idx].x);
            __builtin_nontemporal_store(r.y, &oc[idx].y);
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

hipError_t wilson_apply(const Geom &g, bool fp64, const void *Ul, double kappa, const void *in,
                        void *out, int nb, bool dagger, hipStream_t st, const ApiOut *api) {
    if (nb < 1 || nb > 16) return hipErrorInvalidValue;
    if (api && (!api->y || api->c0 < 0 || api->m < api->c0 + nb)) return hipErrorInvalidValue;
    const ApiOut ao = api ? *api : ApiOut{nullptr, 0, 0};
    const dim3 grid((unsigned)lockstep_blocks(g));
    const dim3 block(64 * nb);
    const ResidOut none{nullptr, nullptr, 0.0, nullptr};
    const BlockOrder lo = lockstep_order(g);
#define DSBCG_L(R, D, MT, GLB)                                                                      \
    hipLaunchKernelGGL((wilson_cm_kernel<R, D, false, MT, GLB>), grid, block, 0, st, g, (const cx<R> *)Ul, \
                       (R)kappa, (const cx<R> *)in, (cx<R> *)out, nb, none, lo, ao)
#define DSBCG_W(R, D)                                                                               \
    do {                                                                                            \
        if (small_bound(nb)) DSBCG_L(R, D, 512, false);                                             \
        else DSBCG_L(R, D, 1024, false);                                                            \
    } while (0)
    if (fp64 && global_links(fp64, nb)) {
        // 5 to 7 columns (at most 448 threads)
        if (dagger) DSBCG_L(double, true, 512, true);
        else DSBCG_L(double, false, 512, true);
    } else if (fp64) {
        if (dagger) DSBCG_W(double, true);
        else DSBCG_W(double, false);
    } else {
        if (dagger) DSBCG_W(float, true);
        else DSBCG_W(float, false);
    }
#undef DSBCG_W
#undef DSBCG_L
    return hipGetLastError();
}

int wilson_resid_workgroups(const Geom &g) { return lockstep_blocks(g); }

hipError_t wilson_resid_norms(const Geom &g, const void *Ul, double kappa, const void *in, const void *b,
                              const void *x, double sigma, int nb, double *partials, hipStream_t st) {
    if (nb < 1 || nb > 16 || !partials) return hipErrorInvalidValue;
    // the partial of a workgroup with no sites is zero
    const dim3 grid((unsigned)wilson_resid_workgroups(g));
    const dim3 block(64 * nb);
    const ResidOut ro{(const zd *)b, (const zd *)x, sigma, partials};
    const BlockOrder lo = lockstep_order(g);
    const ApiOut ao{nullptr, 0, 0};
    if (global_links(true, nb))
        hipLaunchKernelGGL((wilson_cm_kernel<double, true, true, 512, true>), grid, block, 0, st, g,
                           (const zd *)Ul, kappa, (const zd *)in, (zd *)nullptr, nb, ro, lo, ao);
    else if (small_bound(nb))
        hipLaunchKernelGGL((wilson_cm_kernel<double, true, true, 512, false>), grid, block, 0, st, g,
                           (const zd *)Ul, kappa, (const zd *)in, (zd *)nullptr, nb, ro, lo, ao);
    else
        hipLaunchKernelGGL((wilson_cm_kernel<double, true, true, 1024, false>), grid, block, 0, st, g,
                           (const zd *)Ul, kappa, (const zd *)in, (zd *)nullptr, nb, ro, lo, ao);
    return hipGetLastError();
}

// out[c] = sum over workgroups w < nwg of partials[c * nwg + w], c < nb, in a
// fixed order (one block per column).
__global__ __launch_bounds__(256) void sum_columns_kernel(const double *__restrict__ partials, int nwg,
                                                          double *__restrict__ out) {
    __shared__ double red[256];
    const int c = blockIdx.x;
    const double *p = partials + (int64_t)c * nwg;
    double s = 0.0;
    for (int w = threadIdx.x; w < nwg; w += 256) s += p[w];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

hipError_t sum_columns(const double *partials, int nwg, int nb, double *out, hipStream_t st) {
    if (nb < 1 || nb > 16 || nwg < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sum_columns_kernel, dim3(nb), dim3(256), 0, st, partials, nwg, out);
    return hipGetLastError();
}

hipError_t neighbor_table(const Geom &g, int32_t *dev_out, hipStream_t st) {
    hipLaunchKernelGGL(neighbor_kernel, dim3((g.V + 255) / 256), dim3(256), 0, st, g, dev_out);
    return hipGetLastError();
}

// Links [V][4][3][3] (site-major, 36 complex per site) to structure-of-arrays
// [mu*9 + e][V]: 64 sites per workgroup pass through LDS, read as one
// contiguous 36-complex-per-site block and written as 36 runs of 64 sites.
// The LDS rows are padded to 37 complex so that the column reads of a wave
// fall in distinct banks.
template <typename To>
__global__ __launch_bounds__(256) void links_soa_kernel(int64_t V, const zd *__restrict__ U,
                                                        cx<To> *__restrict__ out) {
    constexpr int kSites = 64, kRow = 37;
    __shared__ zd tile[kSites * kRow];
    const int64_t x0 = (int64_t)blockIdx.x * kSites;
    const int ns = (int)min((int64_t)kSites, V - x0);
    const zd *src = U + x0 * 36;
    for (int e = threadIdx.x; e < ns * 36; e += blockDim.x) {
        const int site = e / 36, k = e - site * 36;
        tile[site * kRow + k] = src[e];
    }
    __syncthreads();
    const int site = threadIdx.x & 63;
    if (site >= ns) return;
    for (int k = threadIdx.x >> 6; k < 36; k += 4)
        out[(int64_t)k * V + x0 + site] = cvt<To>(tile[site * kRow + k]);
}

hipError_t links_to_soa(int64_t V, const void *U, void *out, bool fp64, hipStream_t st) {
    const dim3 grid((unsigned)((V + 63) / 64));
    if (fp64)
        hipLaunchKernelGGL((links_soa_kernel<double>), grid, dim3(256), 0, st, V, (const zd *)U,
                           (zd *)out);
    else
        hipLaunchKernelGGL((links_soa_kernel<float>), grid, dim3(256), 0, st, V, (const zd *)U,
                           (zf *)out);
    return hipGetLastError();
}

}  // namespace dsbcg
