// Tall-skinny block kernels of the block Lanczos process and of the
// per-shift recurrences (Sec. 3 of the paper): products V^H W (Gram), block
// combinations W - V alpha - V' beta^H, basis scalings W R^{-1}, and the
// P_j / X_j updates.  All of them stream n x b blocks with b <= 16 and are
// bound by HBM bandwidth.  Blocks are column-major and one thread owns one
// row, so a wave reads 64 consecutive elements of a column.  Gram sums are
// accumulated in FP64 and reduced in a fixed order (bitwise repeatable).

#include "blas.hpp"

namespace dsbcg {

// ---------------------------------------------------------------------------
// Combination out = sum_k X_k C_k, one thread per row.  Coefficients are
// rounded to the data precision and read from LDS with wave-uniform
// addresses.
// ---------------------------------------------------------------------------
template <typename R, int BO>
__device__ inline void combine_row(const TsArgs &a, const cx<R> (*coef)[kMaxW * kMaxW], int64_t row,
                                   cx<R> out[BO]) {
#pragma unroll
    for (int q = 0; q < BO; ++q) out[q] = mk<R>(0, 0);
    for (int k = 0; k < a.K; ++k) {
        const cx<R> *X = (const cx<R> *)a.X[k] + row;
        const int64_t cs = a.cs[k];
        if (a.C[k] == nullptr) {
#pragma unroll
            for (int q = 0; q < BO; ++q)
                if (q < a.bout) out[q] = out[q] + X[q * cs];
        } else {
            for (int p = 0; p < a.bx[k]; ++p) {
                const cx<R> x = X[p * cs];
#pragma unroll
                for (int q = 0; q < BO; ++q)
                    if (q < a.bout) cmac(out[q], x, coef[k][p * kMaxW + q]);
            }
        }
    }
}

template <typename R>
__device__ inline void load_coefs(const TsArgs &a, cx<R> (*coef)[kMaxW * kMaxW]) {
    for (int k = 0; k < a.K; ++k) {
        if (a.C[k] == nullptr) continue;
        for (int e = threadIdx.x; e < a.bx[k] * a.bout; e += blockDim.x) {
            const int p = e / a.bout, q = e - p * a.bout;
            coef[k][p * kMaxW + q] = cvt<R>(a.C[k][p * 16 + q]);
        }
    }
}

// Gram with B x B accumulators per thread (bl == bout == B).
template <typename R, int B>
__global__ __launch_bounds__(256) void ts_reg_kernel(TsArgs a) {
    __shared__ cx<R> coef[3][kMaxW * kMaxW];
    __shared__ zd red[4][B * B];
    load_coefs<R>(a, coef);
    __syncthreads();
    zd G[B][B];
#pragma unroll
    for (int p = 0; p < B; ++p)
#pragma unroll
        for (int q = 0; q < B; ++q) G[p][q] = mk<double>(0, 0);
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r1 = min(a.nrows, r0 + a.rows_per_wg);
    cx<R> *out = (cx<R> *)a.out;
    for (int64_t row = r0 + threadIdx.x; row < r1; row += 256) {
        cx<R> o[B];
        combine_row<R, B>(a, coef, row, o);
        if (out)
#pragma unroll
            for (int q = 0; q < B; ++q) out[q * a.cso + row] = o[q];
        if (a.gram) {
            cx<R> l[B];
            if (a.gram == 2) {
                const cx<R> *Lp = (const cx<R> *)a.L + row;
#pragma unroll
                for (int p = 0; p < B; ++p) l[p] = Lp[p * a.csl];
            } else {
#pragma unroll
                for (int p = 0; p < B; ++p) l[p] = o[p];
            }
#pragma unroll
            for (int p = 0; p < B; ++p)
#pragma unroll
                for (int q = 0; q < B; ++q) cmac_conj(G[p][q], cvt<double>(l[p]), cvt<double>(o[q]));
        }
    }
    if (!a.gram) return;
    // wave reduction by butterflies, then across the four waves
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < B; ++p)
#pragma unroll
        for (int q = 0; q < B; ++q) {
            zd v = G[p][q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                v.x += __shfl_xor(v.x, off, 64);
                v.y += __shfl_xor(v.y, off, 64);
            }
            if (lane == 0) red[wave][p * B + q] = v;
        }
    __syncthreads();
    if (threadIdx.x < B * B) {
        const int p = threadIdx.x / B, q = threadIdx.x - p * B;
        zd s = red[0][threadIdx.x];
        s = s + red[1][threadIdx.x];
        s = s + red[2][threadIdx.x];
        s = s + red[3][threadIdx.x];
        a.partials[(int64_t)blockIdx.x * 256 + p * 16 + q] = s;
    }
}

// General widths: a tile of rows (one per thread) is staged in LDS
// (column-major) and the Gram is accumulated by 2 x 2 blocks of pairs; with
// 128 threads two halves of the tile are summed separately.
template <typename R>
struct TileRows {
    static constexpr int value = sizeof(R) == 8 ? 64 : 128;
};

template <typename R>
__global__ __launch_bounds__(128) void ts_lds_kernel(TsArgs a) {
    constexpr int kTileRows = TileRows<R>::value;
    __shared__ cx<R> coef[3][kMaxW * kMaxW];
    __shared__ cx<R> so[kMaxW * kTileRows];
    __shared__ cx<R> sl[kMaxW * kTileRows];
    __shared__ zd red[4][64];
    load_coefs<R>(a, coef);
    const int t = threadIdx.x;
    const int bl = (a.gram == 1) ? a.bout : a.bl;
    const int nbq = (a.bout + 1) / 2, nbp = (bl + 1) / 2;
    const int nblk = nbp * nbq;
    const int blk = t & 63, half = t >> 6;
    const int bp = (blk < nblk) ? blk / nbq : 0, bq = (blk < nblk) ? blk - (blk / nbq) * nbq : 0;
    zd G[2][2];
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) G[u][v] = mk<double>(0, 0);
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r1 = min(a.nrows, r0 + a.rows_per_wg);
    cx<R> *out = (cx<R> *)a.out;
    __syncthreads();
    for (int64_t t0 = r0; t0 < r1; t0 += kTileRows) {
        const int64_t row = t0 + t;
        const bool ok = row < r1;
        if (ok) {
            cx<R> o[kMaxW];
            combine_row<R, kMaxW>(a, coef, row, o);
            for (int q = 0; q < a.bout; ++q) {
                if (out) out[q * a.cso + row] = o[q];
                so[q * kTileRows + t] = o[q];
            }
            if (a.gram == 2) {
                const cx<R> *Lp = (const cx<R> *)a.L + row;
                for (int p = 0; p < a.bl; ++p) sl[p * kTileRows + t] = Lp[p * a.csl];
            }
        } else {
            for (int q = 0; q < a.bout; ++q) so[q * kTileRows + t] = mk<R>(0, 0);
            if (a.gram == 2)
                for (int p = 0; p < a.bl; ++p) sl[p * kTileRows + t] = mk<R>(0, 0);
        }
        __syncthreads();
        if (a.gram && blk < nblk) {
            const cx<R> *L = (a.gram == 1) ? so : sl;
            const int p0 = 2 * bp, q0 = 2 * bq;
            const bool p1ok = p0 + 1 < bl, q1ok = q0 + 1 < a.bout;
            for (int r = half * 64; r < half * 64 + 64 && r < kTileRows; ++r) {
                const zd l0 = cvt<double>(L[p0 * kTileRows + r]);
                const zd l1 = p1ok ? cvt<double>(L[(p0 + 1) * kTileRows + r]) : mk<double>(0, 0);
                const zd y0 = cvt<double>(so[q0 * kTileRows + r]);
                const zd y1 = q1ok ? cvt<double>(so[(q0 + 1) * kTileRows + r]) : mk<double>(0, 0);
                cmac_conj(G[0][0], l0, y0);
                cmac_conj(G[0][1], l0, y1);
                cmac_conj(G[1][0], l1, y0);
                cmac_conj(G[1][1], l1, y1);
            }
        }
        __syncthreads();
    }
    if (!a.gram) return;
    // combine the two row halves, then write the blocks
    if (half == 1 && blk < nblk)
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v) red[u * 2 + v][blk] = G[u][v];
    __syncthreads();
    if (half == 0 && blk < nblk) {
        const int p0 = 2 * bp, q0 = 2 * bq;
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v) {
                const int p = p0 + u, q = q0 + v;
                if (p < bl && q < a.bout)
                    a.partials[(int64_t)blockIdx.x * 256 + p * 16 + q] =
                        (blockDim.x > 64) ? G[u][v] + red[u * 2 + v][blk] : G[u][v];
            }
    }
}

hipError_t ts_run(bool fp64, TsArgs a, int max_wg, int *nwg_out, hipStream_t st) {
    const int bl = (a.gram == 1) ? a.bout : a.bl;
    const bool reg = a.gram != 2 ? (a.bout <= 6) : (a.bl == a.bout && a.bout <= 6);
    const int tile = reg ? 256 : (fp64 ? TileRows<double>::value : TileRows<float>::value);
    int64_t tiles = (a.nrows + tile - 1) / tile;
    int nwg = (int)(tiles < max_wg ? tiles : max_wg);
    if (nwg < 1) nwg = 1;
    const int64_t per = (tiles + nwg - 1) / nwg;
    a.rows_per_wg = per * tile;
    nwg = (int)((a.nrows + a.rows_per_wg - 1) / a.rows_per_wg);
    if (nwg < 1) nwg = 1;
    (void)bl;
    if (reg) {
#define DSBCG_TS(R, B) hipLaunchKernelGGL((ts_reg_kernel<R, B>), dim3(nwg), dim3(256), 0, st, a)
        switch (a.bout) {
            case 1: if (fp64) DSBCG_TS(double, 1); else DSBCG_TS(float, 1); break;
            case 2: if (fp64) DSBCG_TS(double, 2); else DSBCG_TS(float, 2); break;
            case 3: if (fp64) DSBCG_TS(double, 3); else DSBCG_TS(float, 3); break;
            case 4: if (fp64) DSBCG_TS(double, 4); else DSBCG_TS(float, 4); break;
            case 5: if (fp64) DSBCG_TS(double, 5); else DSBCG_TS(float, 5); break;
            default: if (fp64) DSBCG_TS(double, 6); else DSBCG_TS(float, 6); break;
        }
#undef DSBCG_TS
    } else {
        if (fp64)
            hipLaunchKernelGGL(ts_lds_kernel<double>, dim3(nwg), dim3(TileRows<double>::value), 0, st, a);
        else
            hipLaunchKernelGGL(ts_lds_kernel<float>, dim3(nwg), dim3(TileRows<float>::value), 0, st, a);
    }
    if (nwg_out) *nwg_out = nwg;
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
// Layout conversion / widening / accumulation of lattice fields.
// ---------------------------------------------------------------------------
struct Strides {
    int64_t site, comp, col, base;
};

__host__ __device__ inline Strides strides_of(const FieldDesc &f, int64_t V) {
    if (f.layout == kApi) return {12 * f.ld, f.ld, 1, f.col0};
    return {1, V, f.ld, 0};
}

template <typename Ti, typename To>
__global__ __launch_bounds__(256) void copy_kernel(int64_t V, int cols, const cx<Ti> *__restrict__ in,
                                                   Strides si, cx<To> *__restrict__ out, Strides so,
                                                   int out_cm, int accumulate, double scale) {
    const int64_t total = V * 12 * cols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        // enumerate so that consecutive threads store consecutive elements
        int64_t x, c, r;
        if (out_cm) {
            x = e % V;
            const int64_t k = e / V;
            c = k % 12;
            r = k / 12;
        } else {
            r = e % cols;
            const int64_t k = e / cols;
            c = k % 12;
            x = k / 12;
        }
        const cx<double> v = cvt<double>(in[si.base + x * si.site + c * si.comp + r * si.col]);
        cx<To> *o = out + so.base + x * so.site + c * so.comp + r * so.col;
        if (accumulate) {
            const cx<double> w = cvt<double>(*o);
            *o = cvt<To>(mk<double>(w.x + scale * v.x, w.y + scale * v.y));
        } else {
            *o = cvt<To>(mk<double>(scale * v.x, scale * v.y));
        }
    }
}

hipError_t copy_field(int64_t V, int cols, FieldDesc in, FieldDesc out, bool accumulate,
                      double scale, hipStream_t st) {
    const int64_t total = V * 12 * cols;
    const int64_t want = (total + 255) / 256;
    const dim3 grid((unsigned)(want < 65536 ? (want > 0 ? want : 1) : 65536));
    const Strides si = strides_of(in, V), so = strides_of(out, V);
    const int ocm = out.layout == kCM, acc = accumulate ? 1 : 0;
#define DSBCG_COPY(TI, TO)                                                                   \
    hipLaunchKernelGGL((copy_kernel<TI, TO>), grid, dim3(256), 0, st, V, cols,               \
                       (const cx<TI> *)in.p, si, (cx<TO> *)out.p, so, ocm, acc, scale)
    if (in.fp64 && out.fp64)
        DSBCG_COPY(double, double);
    else if (in.fp64)
        DSBCG_COPY(double, float);
    else if (out.fp64)
        DSBCG_COPY(float, double);
    else
        DSBCG_COPY(float, float);
#undef DSBCG_COPY
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Window update of the per-shift iterates: a workgroup owns 64 rows; the rows
// of the K window blocks are staged in LDS once and each of the four waves
// applies them to every fourth shift, so X_j and P_j rows are read and
// written once per window instead of once per block step.
// ---------------------------------------------------------------------------
template <typename R>
struct WinCols {
    static constexpr int value = sizeof(R) == 8 ? kWinCols64 : kWinCols32;
};

template <typename R, int BC, int MC>
__global__ __launch_bounds__(256) void window_kernel(WinArgs a) {
    constexpr int kRows = 64;
    __shared__ cx<R> vt[WinCols<R>::value * kRows];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kRows;
    const int64_t row = r0 + lane;
    const bool ok = row < a.nrows;
    const int64_t n = a.nrows;
    // stage the window rows: column c of the concatenated window at vt[c * 64 + lane]
    {
        int c0 = 0;
        for (int u = 0; u < a.K; ++u) {
            const cx<R> *Vu = (const cx<R> *)a.Vw[u];
            for (int q = wave; q < a.wb[u]; q += 4)
                vt[(c0 + q) * kRows + lane] = ok ? Vu[(int64_t)q * n + row] : mk<R>(0, 0);
            c0 += a.wb[u];
        }
    }
    __syncthreads();
    if (!ok) return;
    const cx<R> *G = (const cx<R> *)a.G, *Fp = (const cx<R> *)a.Fp;
    const cx<R> *H = (const cx<R> *)a.H, *F = (const cx<R> *)a.F;
    for (int js = wave; js < a.nshift; js += 4) {
        const int j = a.shifts[js];
        const uint32_t xm = a.xmask[j];
        const int cnt = a.count[j];
        const bool wp = a.pmask[j] != 0;
        cx<R> dx[MC], pn[BC];
#pragma unroll
        for (int q = 0; q < MC; ++q) dx[q] = mk<R>(0, 0);
#pragma unroll
        for (int q = 0; q < BC; ++q) pn[q] = mk<R>(0, 0);
        if (a.bp0 > 0) {
            const cx<R> *po = (const cx<R> *)a.Pold + j * a.pstride + row;
            const cx<R> *g = G + j * 256, *fp = Fp + j * 256;
            for (int p = 0; p < a.bp0; ++p) {
                const cx<R> v = po[(int64_t)p * n];
#pragma unroll
                for (int q = 0; q < MC; ++q)
                    if (q < a.m) cmac(dx[q], v, fp[p * 16 + q]);
                if (wp)
#pragma unroll
                    for (int q = 0; q < BC; ++q)
                        if (q < a.bend) cmac(pn[q], v, g[p * 16 + q]);
            }
        }
        int c0 = 0;
        for (int u = 0; u < cnt; ++u) {
            const cx<R> *hu = H + ((int64_t)j * kWinMax + u) * 256;
            const cx<R> *fu = F + ((int64_t)j * kWinMax + u) * 256;
            for (int p = 0; p < a.wb[u]; ++p) {
                const cx<R> v = vt[(c0 + p) * kRows + lane];
#pragma unroll
                for (int q = 0; q < MC; ++q)
                    if (q < a.m) cmac(dx[q], v, fu[p * 16 + q]);
                if (wp)
#pragma unroll
                    for (int q = 0; q < BC; ++q)
                        if (q < a.bend) cmac(pn[q], v, hu[p * 16 + q]);
            }
            c0 += a.wb[u];
        }
        cx<R> *xr = (cx<R> *)a.X + j * a.xstride + row;
#pragma unroll
        for (int q = 0; q < MC; ++q)
            if (q < a.m && ((xm >> q) & 1u)) xr[(int64_t)q * n] = xr[(int64_t)q * n] + dx[q];
        if (wp) {
            cx<R> *pw = (cx<R> *)a.Pnew + j * a.pstride + row;
#pragma unroll
            for (int q = 0; q < BC; ++q)
                if (q < a.bend) pw[(int64_t)q * n] = pn[q];
        }
    }
}

hipError_t window_apply(bool fp64, const WinArgs &a, hipStream_t st) {
    if (a.K < 1 || a.K > kWinMax || a.m < 1 || a.m > 16 || a.bend > 16 || a.bp0 > 16)
        return hipErrorInvalidValue;
    int cols = 0;
    for (int u = 0; u < a.K; ++u) cols += a.wb[u];
    if (cols > (fp64 ? kWinCols64 : kWinCols32)) return hipErrorInvalidValue;
    if (a.nrows <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.nrows + 63) / 64));
    const int bc = a.bend <= 4 ? 4 : a.bend <= 8 ? 8 : 16;
    const int mc = a.m <= 4 ? 4 : a.m <= 8 ? 8 : 16;
#define DSBCG_WIN(R, B, M) hipLaunchKernelGGL((window_kernel<R, B, M>), grid, dim3(256), 0, st, a)
#define DSBCG_WIN_M(R, B)                   \
    do {                                    \
        if (mc == 4) DSBCG_WIN(R, B, 4);    \
        else if (mc == 8) DSBCG_WIN(R, B, 8); \
        else DSBCG_WIN(R, B, 16);           \
    } while (0)
#define DSBCG_WIN_B(R)                      \
    do {                                    \
        if (bc == 4) DSBCG_WIN_M(R, 4);     \
        else if (bc == 8) DSBCG_WIN_M(R, 8); \
        else DSBCG_WIN_M(R, 16);            \
    } while (0)
    if (fp64) DSBCG_WIN_B(double);
    else DSBCG_WIN_B(float);
#undef DSBCG_WIN_B
#undef DSBCG_WIN_M
#undef DSBCG_WIN
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
