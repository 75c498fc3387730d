// Tall-skinny block kernels of the block Lanczos process and of the
// per-shift recurrences (Sec. 3 of the paper): products V^H W (Gram), block
// combinations W - V alpha - V' beta^H, basis scalings W R^{-1}, and the
// P_j / X_j updates.  All of them stream n x b blocks with b <= 16 and are
// bound by HBM bandwidth; Gram sums are accumulated in FP64 and reduced in a
// fixed order, so results are bitwise repeatable.

#include "blas.hpp"

namespace dsbcg {

// ---------------------------------------------------------------------------
// Combination + Gram engine.  A workgroup owns a contiguous range of rows and
// walks it in tiles of TR rows: the input tiles are staged in LDS with
// coalesced loads, the combination is formed element-wise from LDS (and
// optionally stored), and the Gram partial sums are accumulated from LDS.
// Inputs may alias the output: a tile is fully read before it is written and
// tiles of different workgroups never overlap.
// ---------------------------------------------------------------------------
template <typename R>
struct TsTile {
    static constexpr int TR = sizeof(R) == 8 ? 32 : 64;
};

template <typename R>
__global__ __launch_bounds__(kTsThreads) void ts_kernel(TsArgs a) {
    constexpr int TR = TsTile<R>::TR;
    __shared__ cx<R> xin[3][TR * kMaxW];
    __shared__ cx<R> otile[TR * kMaxW];
    __shared__ cx<R> ltile[TR * kMaxW];
    __shared__ cx<R> coef[3][kMaxW * kMaxW];
    __shared__ zd red[kTsThreads];

    const int tid = threadIdx.x;
    const int bout = a.bout;
    // coefficients, rounded to the data precision
    for (int k = 0; k < a.K; ++k) {
        if (a.C[k] == nullptr) continue;
        for (int e = tid; e < a.bx[k] * bout; e += kTsThreads) {
            const int p = e / bout, q = e - p * bout;
            coef[k][p * kMaxW + q] = cvt<R>(a.C[k][p * 16 + q]);
        }
    }

    const int pairs = a.gram ? (a.gram == 1 ? bout : a.bl) * bout : 0;
    const int groups = pairs ? kTsThreads / pairs : 0;
    const int grp = pairs ? tid / pairs : 0;
    const int pr = pairs ? tid - grp * pairs : 0;
    const int gp = pairs ? pr / bout : 0, gq = pairs ? pr - gp * bout : 0;
    zd acc = mk<double>(0, 0);

    const int64_t r_begin = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r_end = min(a.nrows, r_begin + a.rows_per_wg);
    __syncthreads();

    for (int64_t t0 = r_begin; t0 < r_end; t0 += TR) {
        const int nr = (int)min((int64_t)TR, r_end - t0);
        // stage the input tiles
        for (int k = 0; k < a.K; ++k) {
            const cx<R> *X = (const cx<R> *)a.X[k];
            const int bx = a.bx[k];
            const int64_t ld = a.ldx[k];
            for (int e = tid; e < nr * bx; e += kTsThreads) {
                const int r = e / bx, p = e - r * bx;
                xin[k][r * kMaxW + p] = X[(t0 + r) * ld + p];
            }
        }
        if (a.gram == 2) {
            const cx<R> *Lp = (const cx<R> *)a.L;
            for (int e = tid; e < nr * a.bl; e += kTsThreads) {
                const int r = e / a.bl, p = e - r * a.bl;
                ltile[r * kMaxW + p] = Lp[(t0 + r) * a.ldl + p];
            }
        }
        __syncthreads();
        // combination
        cx<R> *out = (cx<R> *)a.out;
        for (int e = tid; e < nr * bout; e += kTsThreads) {
            const int r = e / bout, q = e - r * bout;
            cx<R> v = mk<R>(0, 0);
            for (int k = 0; k < a.K; ++k) {
                if (a.C[k] == nullptr) {
                    v = v + xin[k][r * kMaxW + q];
                } else {
                    for (int p = 0; p < a.bx[k]; ++p)
                        cmac(v, xin[k][r * kMaxW + p], coef[k][p * kMaxW + q]);
                }
            }
            otile[r * kMaxW + q] = v;
            if (out) out[(t0 + r) * a.ldo + q] = v;
        }
        __syncthreads();
        // Gram partial sums in FP64
        if (pairs && grp < groups) {
            const cx<R> *lt = (a.gram == 1) ? otile : ltile;
            for (int r = grp; r < nr; r += groups)
                cmac_conj(acc, cvt<double>(lt[r * kMaxW + gp]), cvt<double>(otile[r * kMaxW + gq]));
        }
        __syncthreads();
    }

    if (pairs) {
        red[tid] = acc;
        __syncthreads();
        if (tid < pairs) {
            zd s = red[tid];
            for (int g = 1; g < groups; ++g) s = s + red[g * pairs + tid];
            a.partials[(int64_t)blockIdx.x * 256 + gp * 16 + gq] = s;
        }
    }
}

hipError_t ts_run(bool fp64, TsArgs a, int nwg, hipStream_t st) {
    if (fp64)
        hipLaunchKernelGGL(ts_kernel<double>, dim3(nwg), dim3(kTsThreads), 0, st, a);
    else
        hipLaunchKernelGGL(ts_kernel<float>, dim3(nwg), dim3(kTsThreads), 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void reduce_kernel(const zd *__restrict__ partials, int nwg,
                                                     zd *__restrict__ out) {
    __shared__ zd red[256];
    const int e = blockIdx.x;  // element index p*16+q
    zd s = mk<double>(0, 0);
    for (int w = threadIdx.x; w < nwg; w += 256) s = s + partials[(int64_t)w * 256 + e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = red[0];
}

hipError_t reduce_partials(const zd *partials, int nwg, int nelem, zd *out, hipStream_t st) {
    hipLaunchKernelGGL(reduce_kernel, dim3(nelem), dim3(256), 0, st, partials, nwg, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Layout conversion / widening / accumulation.
// ---------------------------------------------------------------------------
template <typename Ti, typename To>
__global__ __launch_bounds__(256) void copy_kernel(int64_t V, int cols, const cx<Ti> *__restrict__ in,
                                                   int64_t in_ld, int in_order, int in_col0,
                                                   cx<To> *__restrict__ out, int64_t out_ld,
                                                   int out_order, int accumulate, double scale) {
    const int64_t total = V * 12 * cols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        // enumerate in the output's row order so that stores are contiguous
        const int64_t orow = e / cols;
        const int col = (int)(e - orow * cols);
        int64_t x, c;
        if (out_order == kApi) {
            x = orow / 12;
            c = orow - x * 12;
        } else {
            c = orow / V;
            x = orow - c * V;
        }
        const int64_t irow = (in_order == kApi) ? x * 12 + c : c * V + x;
        const cx<double> v = cvt<double>(in[irow * in_ld + in_col0 + col]);
        cx<To> *o = out + orow * out_ld + col;
        if (accumulate) {
            const cx<double> w = cvt<double>(*o);
            *o = cvt<To>(mk<double>(w.x + scale * v.x, w.y + scale * v.y));
        } else {
            *o = cvt<To>(mk<double>(scale * v.x, scale * v.y));
        }
    }
}

hipError_t copy_field(bool in_fp64, bool out_fp64, int64_t V, int cols, const void *in,
                      int64_t in_ld, int in_order, int in_col0, void *out, int64_t out_ld,
                      int out_order, bool accumulate, double scale, hipStream_t st) {
    const int64_t total = V * 12 * cols;
    const int64_t want = (total + 255) / 256;
    const dim3 grid((unsigned)(want < 65536 ? (want > 0 ? want : 1) : 65536));
    const int acc = accumulate ? 1 : 0;
#define DSBCG_COPY(TI, TO)                                                                   \
    hipLaunchKernelGGL((copy_kernel<TI, TO>), grid, dim3(256), 0, st, V, cols,               \
                       (const cx<TI> *)in, in_ld, in_order, in_col0, (cx<TO> *)out, out_ld, \
                       out_order, acc, scale)
    if (in_fp64 && out_fp64)
        DSBCG_COPY(double, double);
    else if (in_fp64)
        DSBCG_COPY(double, float);
    else if (out_fp64)
        DSBCG_COPY(float, double);
    else
        DSBCG_COPY(float, float);
#undef DSBCG_COPY
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-shift update, one thread per row.  The coefficient matrices are read
// with wave-uniform addresses (scalar loads); the basis row V_i is read once
// from HBM and re-read from cache for every further shift.
// ---------------------------------------------------------------------------
template <typename R, int BC>
__global__ __launch_bounds__(256) void shift_kernel(ShiftArgs a) {
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row >= a.nrows) return;
    const cx<R> *__restrict__ V = (const cx<R> *)a.V;
    const cx<R> *__restrict__ Nc = (const cx<R> *)a.N;
    const cx<R> *__restrict__ Mc = (const cx<R> *)a.M;
    const int b = a.b, bp = a.bp, m = a.m;
    for (int js = 0; js < a.nshift; ++js) {
        const int j = a.shifts[js];
        const uint32_t mask = a.colmask[j];
        cx<R> pn[BC];
        const cx<R> *vr = V + row * b;
#pragma unroll
        for (int q = 0; q < BC; ++q)
            if (q < b) pn[q] = vr[q];
        if (!a.first) {
            const cx<R> *po = (const cx<R> *)a.Pold + j * a.pstride + row * bp;
            const cx<R> *Nj = Nc + j * 256;
            for (int p = 0; p < bp; ++p) {
                const cx<R> v = po[p];
#pragma unroll
                for (int q = 0; q < BC; ++q)
                    if (q < b) {
                        const cx<R> nn = Nj[p * 16 + q];
                        pn[q].x = fma(-v.x, nn.x, pn[q].x);
                        pn[q].x = fma(v.y, nn.y, pn[q].x);
                        pn[q].y = fma(-v.x, nn.y, pn[q].y);
                        pn[q].y = fma(-v.y, nn.x, pn[q].y);
                    }
            }
        }
        cx<R> *pw = (cx<R> *)a.Pnew + j * a.pstride + row * b;
#pragma unroll
        for (int q = 0; q < BC; ++q)
            if (q < b) pw[q] = pn[q];
        cx<R> *xr = (cx<R> *)a.X + j * a.xstride + row * m;
        const cx<R> *Mj = Mc + j * 256;
        for (int l = 0; l < m; ++l) {
            if (!((mask >> l) & 1u)) continue;
            cx<R> x = xr[l];
#pragma unroll
            for (int q = 0; q < BC; ++q)
                if (q < b) cmac(x, pn[q], Mj[q * 16 + l]);
            xr[l] = x;
        }
    }
}

hipError_t shift_update(bool fp64, const ShiftArgs &a, hipStream_t st) {
    const dim3 grid((unsigned)((a.nrows + 255) / 256));
    const int bc = a.b <= 4 ? 4 : a.b <= 8 ? 8 : a.b <= 12 ? 12 : 16;
#define DSBCG_SHIFT(R, N) hipLaunchKernelGGL((shift_kernel<R, N>), grid, dim3(256), 0, st, a)
    if (fp64) {
        if (bc == 4) DSBCG_SHIFT(double, 4);
        else if (bc == 8) DSBCG_SHIFT(double, 8);
        else if (bc == 12) DSBCG_SHIFT(double, 12);
        else DSBCG_SHIFT(double, 16);
    } else {
        if (bc == 4) DSBCG_SHIFT(float, 4);
        else if (bc == 8) DSBCG_SHIFT(float, 8);
        else if (bc == 12) DSBCG_SHIFT(float, 12);
        else DSBCG_SHIFT(float, 16);
    }
#undef DSBCG_SHIFT
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void nonfinite_kernel(const double *__restrict__ d, int64_t count,
                                                        int32_t *flag) {
    bool bad = false;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(d[e]);
    if (bad) atomicOr(flag, 1);
}

hipError_t find_nonfinite(const double *data, int64_t count, int32_t *flag, hipStream_t st) {
    const int64_t want = (count + 255) / 256;
    const dim3 grid((unsigned)(want < 16384 ? (want > 0 ? want : 1) : 16384));
    hipLaunchKernelGGL(nonfinite_kernel, grid, dim3(256), 0, st, data, count, flag);
    return hipGetLastError();
}

}  // namespace dsbcg
