// Tall-skinny block kernels of the block Lanczos process and of the
// per-shift recurrences (Sec. 3 of the paper): products V^H W (Gram), block
// combinations W - V alpha - V' beta^H, basis scalings W R^{-1}, and the
// windowed P_j / X_j updates (matrix cores).  All of them stream n x b blocks with b <= 16 and are
// bound by HBM bandwidth.  Blocks are column-major and one thread owns one
// row, so a wave reads 64 consecutive elements of a column.  Gram sums are
// accumulated in FP64 and reduced in a fixed order (bitwise repeatable).

#include "blas.hpp"

#include <algorithm>

namespace dsbcg {

// ---------------------------------------------------------------------------
// Combination out = sum_k X_k C_k and Gram products, one thread per row.
// Widths are compile-time (B) so that every load of a row is issued before
// the arithmetic that uses it; columns past a block's width are read at its
// last column and meet zero coefficients.  Coefficients are rounded to the
// data precision and read from LDS with wave-uniform addresses; C_k == NULL
// means the identity.
// ---------------------------------------------------------------------------
template <typename R, int B>
__device__ inline void load_coefs(const TsArgs &a, cx<R> *coef) {
    for (int e = threadIdx.x; e < 3 * B * B; e += blockDim.x) {
        const int k = e / (B * B), r = e - k * B * B, p = r / B, q = r - p * B;
        cx<R> v = mk<R>(0, 0);
        if (k < a.K && p < a.bx[k] && q < a.bout)
            v = a.C[k] ? cvt<R>(a.C[k][p * 16 + q]) : (p == q ? mk<R>(1, 0) : mk<R>(0, 0));
        coef[e] = v;
    }
}

template <typename R, int B, int K>
__device__ inline void combine_row(const TsArgs &a, const cx<R> *coef, int64_t row, cx<R> o[B]) {
#pragma unroll
    for (int q = 0; q < B; ++q) o[q] = mk<R>(0, 0);
    if (B <= 8) {
        // every input row in flight at once
        cx<R> x[K][B];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            // inputs k >= a.K have no block (NULL) and zero coefficients
            if (k < a.K) {
                const cx<R> *X = (const cx<R> *)a.X[k] + row;
                const int last = max(a.bx[k] - 1, 0);
#pragma unroll
                for (int p = 0; p < B; ++p) x[k][p] = X[(int64_t)min(p, last) * a.cs[k]];
            } else {
#pragma unroll
                for (int p = 0; p < B; ++p) x[k][p] = mk<R>(0, 0);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int p = 0; p < B; ++p) {
                // one coefficient row at a time (all of them at once would
                // need 4 K B^2 registers)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < B; ++q) cmac(o[q], x[k][p], coef[(k * B + p) * B + q]);
            }
    } else {
        // wide blocks: one input block at a time (only the a.K inputs that exist)
        const int nk = min(K, a.K);
#pragma unroll 1
        for (int k = 0; k < nk; ++k) {
            const cx<R> *X = (const cx<R> *)a.X[k] + row;
            const int last = max(a.bx[k] - 1, 0);
            cx<R> x[B];
#pragma unroll
            for (int p = 0; p < B; ++p) x[p] = X[(int64_t)min(p, last) * a.cs[k]];
#pragma unroll
            for (int p = 0; p < B; ++p) {
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < B; ++q) cmac(o[q], x[p], coef[(k * B + p) * B + q]);
            }
        }
    }
}

// Rows per thread.  FP32: two consecutive rows, loaded and stored as one
// 16-byte vector (row counts, column strides and block bases are even).
// FP64: one row (already a 16-byte access; a second row per thread only
// costs occupancy).
template <typename R>
struct RowGroup;
template <>
struct RowGroup<float> {
    static constexpr int rows = 2;
    static __device__ inline void load(const cx<float> *p, cx<float> v[2]) {
        const float4 w = *(const float4 *)p;
        v[0] = mk<float>(w.x, w.y);
        v[1] = mk<float>(w.z, w.w);
    }
    static __device__ inline void store(cx<float> *p, const cx<float> v[2]) {
        *(float4 *)p = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
    }
};
template <>
struct RowGroup<double> {
    static constexpr int rows = 1;
    static __device__ inline void load(const cx<double> *p, cx<double> v[1]) { v[0] = *p; }
    static __device__ inline void store(cx<double> *p, const cx<double> v[1]) { *p = v[0]; }
};

// combine_row for a group of RPT consecutive rows (widths B <= 8): every
// input in flight at once, one coefficient row at a time.
template <typename R, int B, int K, int RPT>
__device__ inline void combine_rows(const TsArgs &a, const cx<R> *coef, int64_t row, cx<R> o[RPT][B]) {
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int q = 0; q < B; ++q) o[i][q] = mk<R>(0, 0);
    cx<R> x[K][B][RPT];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (k < a.K) {
            const cx<R> *X = (const cx<R> *)a.X[k] + row;
            const int last = max(a.bx[k] - 1, 0);
#pragma unroll
            for (int p = 0; p < B; ++p) RowGroup<R>::load(X + (int64_t)min(p, last) * a.cs[k], x[k][p]);
        } else {
#pragma unroll
            for (int p = 0; p < B; ++p)
#pragma unroll
                for (int i = 0; i < RPT; ++i) x[k][p][i] = mk<R>(0, 0);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int p = 0; p < B; ++p) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < B; ++q) {
                const cx<R> c = coef[(k * B + p) * B + q];
#pragma unroll
                for (int i = 0; i < RPT; ++i) cmac(o[i][q], x[k][p][i], c);
            }
        }
}

// Register Gram: GRAM 0 none, 1 out^H out (upper triangle, mirrored), 2 L^H out,
// 3 the diagonal of out^H out only (column norms), 4 both L^H out and
// out^H out (widths up to 5).  At width 5 the 40 complex FP64 accumulators
// of gram 4 hold the kernel at one wave per SIMD; measured at 32^3 x 64 this
// is faster than splitting the two blocks over a pair of waves that read the
// same rows (165 against 136 ms of Gram/update kernels per FP64 solve) and
// than a two-waves bound that spills (141 ms).  K inputs.
template <typename R, int B, int K, int GRAM>
__global__ __launch_bounds__(256) void ts_reg_kernel(TsArgs a) {
    if (a.skip && *a.skip) return;  // uniform: before any barrier
    __shared__ cx<R> coef[3 * B * B];
    __shared__ zd red[4][B * B];
    load_coefs<R, B>(a, coef);
    __syncthreads();
    constexpr int NG = GRAM == 0 ? 1 : B * B;
    constexpr int NG2 = GRAM == 4 ? B * B : 1;  // out^H out next to L^H out
    zd G[NG], G2[NG2];
#pragma unroll
    for (int e = 0; e < NG; ++e) G[e] = mk<double>(0, 0);
#pragma unroll
    for (int e = 0; e < NG2; ++e) G2[e] = mk<double>(0, 0);
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r1 = min(a.nrows, r0 + a.rows_per_wg);
    cx<R> *out = (cx<R> *)a.out;
    const int bl = (GRAM == 2 || GRAM == 4) ? a.bl : 0;
    constexpr int RPT = RowGroup<R>::rows;
#pragma unroll 1
    for (int64_t row = r0 + RPT * threadIdx.x; row < r1; row += 256 * RPT) {
        cx<R> l[B][RPT];
        if (GRAM == 2 || GRAM == 4) {
            const cx<R> *Lp = (const cx<R> *)a.L + row;
#pragma unroll
            for (int p = 0; p < B; ++p) {
                RowGroup<R>::load(Lp + (int64_t)min(p, bl - 1) * a.csl, l[p]);
                if (p >= bl)
#pragma unroll
                    for (int i = 0; i < RPT; ++i) l[p][i] = mk<R>(0, 0);
            }
        }
        cx<R> o[RPT][B];
        combine_rows<R, B, K, RPT>(a, coef, row, o);
        if (out)
#pragma unroll
            for (int q = 0; q < B; ++q)
                if (q < a.bout) {
                    cx<R> v[RPT];
#pragma unroll
                    for (int i = 0; i < RPT; ++i) v[i] = o[i][q];
                    RowGroup<R>::store(out + q * a.cso + row, v);
                }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            if (GRAM == 1) {
                zd od[B];
#pragma unroll
                for (int q = 0; q < B; ++q) od[q] = cvt<double>(o[i][q]);
#pragma unroll
                for (int p = 0; p < B; ++p)
#pragma unroll
                    for (int q = p; q < B; ++q) cmac_conj(G[p * B + q], od[p], od[q]);
            } else if (GRAM == 3) {
#pragma unroll
                for (int q = 0; q < B; ++q) G[q * B + q].x += norm2(cvt<double>(o[i][q]));
            } else if (GRAM == 2 || GRAM == 4) {
                zd od[B];
#pragma unroll
                for (int q = 0; q < B; ++q) od[q] = cvt<double>(o[i][q]);
#pragma unroll
                for (int p = 0; p < B; ++p) {
                    const zd lp = cvt<double>(l[p][i]);
#pragma unroll
                    for (int q = 0; q < B; ++q) cmac_conj(G[p * B + q], lp, od[q]);
                }
                if (GRAM == 4)
#pragma unroll
                    for (int p = 0; p < B; ++p)
#pragma unroll
                        for (int q = p; q < B; ++q) cmac_conj(G2[p * B + q], od[p], od[q]);
            }
        }
    }
    if (GRAM == 0) return;
    // wave reduction by butterflies, then across the four waves; GRAM 4 runs
    // this twice (L^H out into entries 0..255 of the workgroup's partials,
    // then out^H out into 256..511)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int part = 0; part < (GRAM == 4 ? 2 : 1); ++part) {
        const int gm = GRAM == 4 ? (part ? 1 : 2) : GRAM;  // the mode of this part
        if (part) __syncthreads();                          // red is reused
#pragma unroll
        for (int p = 0; p < B; ++p)
#pragma unroll
            for (int q = 0; q < B; ++q) {
                if ((gm == 1 && q < p) || (gm == 3 && q != p)) continue;
                zd v = (GRAM == 4 && part) ? G2[(p * B + q) % NG2] : G[p * B + q];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    v.x += __shfl_xor(v.x, off, 64);
                    v.y += __shfl_xor(v.y, off, 64);
                }
                if (lane == 0) red[wave][p * B + q] = v;
            }
        __syncthreads();
        if (threadIdx.x < B * B) {
            int p = threadIdx.x / B, q = threadIdx.x - p * B;
            const bool mirror = gm == 1 && q < p;
            const int e = mirror ? q * B + p : p * B + q;
            zd s = mk<double>(0, 0);
            if (gm != 3 || p == q) {
                s = red[0][e];
                s = s + red[1][e];
                s = s + red[2][e];
                s = s + red[3][e];
            }
            a.partials[(int64_t)blockIdx.x * kPartialStride + 256 * part + p * 16 + q] = mirror ? conj(s) : s;
        }
    }
}

// Wider blocks (B = 16): a workgroup of 4 waves takes tiles of 64 rows.
// Each row's outputs are formed by 4 threads (output columns q = c, c + 4,
// c + 8, c + 12 for thread group c) and staged in LDS, column-major with
// rows padded to 65 entries so that the Gram reads of different columns
// fall in different banks.  The Gram is accumulated by 2 x 2 blocks of
// pairs, each block by 4 threads over a quarter of the tile's rows, and the
// quarters are added in a fixed order at the end.
template <typename R>
struct TileRows {
    static constexpr int value = 64;
};
constexpr int kLdsThreads = 256;

template <typename R>
__global__ __launch_bounds__(kLdsThreads) void ts_lds_kernel(TsArgs a) {
    if (a.skip && *a.skip) return;  // uniform: before any barrier
    constexpr int B = kMaxW;
    constexpr int kTileRows = TileRows<R>::value;
    constexpr int kLd = kTileRows + 1;      // padded column length in LDS
    constexpr int kQuarter = kTileRows / 4;
    constexpr size_t kTileBytes = 2 * (size_t)B * kLd * sizeof(cx<R>);
    constexpr size_t kRedBytes = 4 * 8 * 64 * sizeof(zd);
    __shared__ cx<R> coef[3 * B * B];
    // so and sl (the tile's outputs and L columns) while the tiles run, the
    // quarters' partial Gram blocks afterwards
    __shared__ __align__(16) char lds[kTileBytes > kRedBytes ? kTileBytes : kRedBytes];
    cx<R> *so = reinterpret_cast<cx<R> *>(lds);
    cx<R> *sl = so + B * kLd;
    load_coefs<R, B>(a, coef);
    const int t = threadIdx.x;
    const bool withL = a.gram == 2 || a.gram == 4;  // gram 4: a.bl == a.bout (checked by ts_run)
    const int bl = withL ? a.bl : a.bout;           // gram 3 (diagonal) runs as gram 1
    const int nbq = (a.bout + 1) / 2, nbp = (bl + 1) / 2;
    const int nblk = nbp * nbq;
    const int lane = t & 63, grp = t >> 6;         // combination: row lane, column group
    const int blk = lane, quarter = grp;           // Gram: 2 x 2 block, quarter of the rows
    const int bp = (blk < nblk) ? blk / nbq : 0, bq = (blk < nblk) ? blk - (blk / nbq) * nbq : 0;
    zd G[2][2], G2[2][2];  // G2: out^H out of gram 4
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) G[u][v] = G2[u][v] = mk<double>(0, 0);
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r1 = min(a.nrows, r0 + a.rows_per_wg);
    cx<R> *out = (cx<R> *)a.out;
    __syncthreads();
    for (int64_t t0 = r0; t0 < r1; t0 += kTileRows) {
        __asm__ volatile("" ::: "memory");
        const int64_t row = t0 + lane;
        const bool ok = row < r1;
        // outputs q = grp + 4 j of this row: out = sum_k X_k C_k, every input
        // of a block in flight at once (past bx[k] the coefficients are
        // zero), in the order of combine_row
        cx<R> o[B / 4];
#pragma unroll
        for (int j = 0; j < B / 4; ++j) o[j] = mk<R>(0, 0);
        if (ok) {
#pragma unroll 1
            for (int k = 0; k < a.K; ++k) {
                const cx<R> *X = (const cx<R> *)a.X[k] + row;
                const int last = max(a.bx[k] - 1, 0);
                cx<R> x[B];
#pragma unroll
                for (int p = 0; p < B; ++p) x[p] = X[(int64_t)min(p, last) * a.cs[k]];
#pragma unroll
                for (int p = 0; p < B; ++p) {
                    // one coefficient row at a time
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int j = 0; j < B / 4; ++j) cmac(o[j], x[p], coef[(k * B + p) * B + grp + 4 * j]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < B / 4; ++j) {
            const int q = grp + 4 * j;
            if (ok && out && q < a.bout) out[q * a.cso + row] = o[j];
            so[q * kLd + lane] = (ok && q < a.bout) ? o[j] : mk<R>(0, 0);
            if (withL) {
                cx<R> v = mk<R>(0, 0);
                if (ok && q < a.bl) v = ((const cx<R> *)a.L)[(int64_t)q * a.csl + row];
                sl[q * kLd + lane] = v;
            }
        }
        __syncthreads();
        if (a.gram && blk < nblk) {
            const cx<R> *L = withL ? sl : so;
            const int p0 = 2 * bp, q0 = 2 * bq;
#pragma unroll 2
            for (int r = quarter * kQuarter; r < (quarter + 1) * kQuarter; ++r) {
                const zd l0 = cvt<double>(L[p0 * kLd + r]);
                const zd l1 = cvt<double>(L[(p0 + 1) * kLd + r]);
                const zd y0 = cvt<double>(so[q0 * kLd + r]);
                const zd y1 = cvt<double>(so[(q0 + 1) * kLd + r]);
                cmac_conj(G[0][0], l0, y0);
                cmac_conj(G[0][1], l0, y1);
                cmac_conj(G[1][0], l1, y0);
                cmac_conj(G[1][1], l1, y1);
                if (a.gram == 4) {
                    const zd o0 = cvt<double>(so[p0 * kLd + r]);
                    const zd o1 = cvt<double>(so[(p0 + 1) * kLd + r]);
                    cmac_conj(G2[0][0], o0, y0);
                    cmac_conj(G2[0][1], o0, y1);
                    cmac_conj(G2[1][0], o1, y0);
                    cmac_conj(G2[1][1], o1, y1);
                }
            }
        }
        __syncthreads();
    }
    if (!a.gram) return;
    // add the four quarters in a fixed order, then write the blocks
    zd *red = reinterpret_cast<zd *>(lds);  // [quarter][8][64]
    if (blk < nblk)
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v) {
                red[(quarter * 8 + u * 2 + v) * 64 + blk] = G[u][v];
                red[(quarter * 8 + 4 + u * 2 + v) * 64 + blk] = G2[u][v];
            }
    __syncthreads();
    if (quarter == 0 && blk < nblk) {
        const int p0 = 2 * bp, q0 = 2 * bq;
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v) {
                const int p = p0 + u, q = q0 + v;
                if (p < bl && q < a.bout) {
                    zd g = red[(u * 2 + v) * 64 + blk], g2 = red[(4 + u * 2 + v) * 64 + blk];
                    for (int h = 1; h < 4; ++h) {
                        g = g + red[(h * 8 + u * 2 + v) * 64 + blk];
                        g2 = g2 + red[(h * 8 + 4 + u * 2 + v) * 64 + blk];
                    }
                    a.partials[(int64_t)blockIdx.x * kPartialStride + p * 16 + q] = g;
                    if (a.gram == 4) a.partials[(int64_t)blockIdx.x * kPartialStride + 256 + p * 16 + q] = g2;
                }
            }
    }
}

template <typename R, int B, int K>
void ts_launch_reg(const TsArgs &a, int nwg, hipStream_t st) {
    // widths 7 and 8 only without a full Gram (register budget)
    if constexpr (B <= 6) {
        if (a.gram == 1) {
            hipLaunchKernelGGL((ts_reg_kernel<R, B, K, 1>), dim3(nwg), dim3(256), 0, st, a);
            return;
        }
        if (a.gram == 2) {
            hipLaunchKernelGGL((ts_reg_kernel<R, B, K, 2>), dim3(nwg), dim3(256), 0, st, a);
            return;
        }
    }
    if constexpr (B <= 5) {
        if (a.gram == 4) {
            hipLaunchKernelGGL((ts_reg_kernel<R, B, K, 4>), dim3(nwg), dim3(256), 0, st, a);
            return;
        }
    }
    if (a.gram == 3)
        hipLaunchKernelGGL((ts_reg_kernel<R, B, K, 3>), dim3(nwg), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((ts_reg_kernel<R, B, K, 0>), dim3(nwg), dim3(256), 0, st, a);
}

template <typename R, int B>
void ts_launch_k(const TsArgs &a, int nwg, hipStream_t st) {
    if (a.K == 1) ts_launch_reg<R, B, 1>(a, nwg, st);
    else if (a.K == 2) ts_launch_reg<R, B, 2>(a, nwg, st);
    else ts_launch_reg<R, B, 3>(a, nwg, st);
}

template <typename R>
void ts_launch(const TsArgs &a, int w, int nwg, hipStream_t st) {
    switch (w) {
        case 1: ts_launch_k<R, 1>(a, nwg, st); break;
        case 2: ts_launch_k<R, 2>(a, nwg, st); break;
        case 3: ts_launch_k<R, 3>(a, nwg, st); break;
        case 4: ts_launch_k<R, 4>(a, nwg, st); break;
        case 5: ts_launch_k<R, 5>(a, nwg, st); break;
        case 6: ts_launch_k<R, 6>(a, nwg, st); break;
        case 7: ts_launch_k<R, 7>(a, nwg, st); break;
        case 8: ts_launch_k<R, 8>(a, nwg, st); break;
        default:
            hipLaunchKernelGGL(ts_lds_kernel<R>, dim3(nwg), dim3(kLdsThreads), 0, st, a);
            break;
    }
}

hipError_t ts_run(bool fp64, TsArgs a, int max_wg, int *nwg_out, hipStream_t st) {
    if (a.K < 1 || a.K > 3 || a.bout < 1 || a.bout > kMaxW) return hipErrorInvalidValue;
    for (int k = 0; k < a.K; ++k)
        if (a.bx[k] < 0 || a.bx[k] > kMaxW) return hipErrorInvalidValue;
    if ((a.gram == 2 || a.gram == 4) && (a.bl < 1 || a.bl > kMaxW)) return hipErrorInvalidValue;
    if (a.gram == 4 && (a.bl != a.bout || a.out)) return hipErrorInvalidValue;
    // register kernel: every input, output and L width within w <= 6, or
    // w <= 8 without a full Gram
    int w = a.bout;
    for (int k = 0; k < a.K; ++k) w = std::max(w, a.bx[k]);
    if (a.gram == 2 || a.gram == 4) w = std::max(w, a.bl);
    // gram 4 keeps two Gram blocks in registers: widths up to 5
    const bool reg = a.gram == 4 ? w <= 5 : (w <= 6 || (w <= 8 && (a.gram == 0 || a.gram == 3)));
    // the FP32 register kernel moves two rows per thread: even row counts,
    // column strides and block offsets
    if (reg && !fp64) {
        if (a.nrows & 1) return hipErrorInvalidValue;
        for (int k = 0; k < a.K; ++k)
            if ((a.cs[k] & 1) || ((uintptr_t)a.X[k] & 15)) return hipErrorInvalidValue;
        if (a.out && ((a.cso & 1) || ((uintptr_t)a.out & 15))) return hipErrorInvalidValue;
        if ((a.gram == 2 || a.gram == 4) && ((a.csl & 1) || ((uintptr_t)a.L & 15))) return hipErrorInvalidValue;
    }
    const int tile = reg ? (fp64 ? 256 : 512) : (fp64 ? TileRows<double>::value : TileRows<float>::value);
    int64_t tiles = (a.nrows + tile - 1) / tile;
    int nwg = (int)(tiles < max_wg ? tiles : max_wg);
    if (nwg < 1) nwg = 1;
    const int64_t per = (tiles + nwg - 1) / nwg;
    a.rows_per_wg = per * tile;
    nwg = (int)((a.nrows + a.rows_per_wg - 1) / a.rows_per_wg);
    if (nwg < 1) nwg = 1;
    if (fp64) ts_launch<double>(a, reg ? w : 16, nwg, st);
    else ts_launch<float>(a, reg ? w : 16, nwg, st);
    if (nwg_out) *nwg_out = nwg;
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void reduce_kernel(const zd *__restrict__ partials, int nwg,
                                                     zd *__restrict__ out) {
    __shared__ zd red[256];
    const int e = blockIdx.x;  // element index p*16+q
    zd s = mk<double>(0, 0);
    for (int w = threadIdx.x; w < nwg; w += 256) s = s + partials[(int64_t)w * kPartialStride + e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = red[0];
}

hipError_t reduce_partials(const zd *partials, int nwg, int nelem, zd *out, hipStream_t st, int off) {
    if (off < 0 || off + nelem > kPartialStride) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reduce_kernel, dim3(nelem), dim3(256), 0, st, partials + off, nwg, out);
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

// Layout change (column-major <-> [V][12][ld]) through an LDS tile of 32
// sites x 12 components x up to 8 columns: the tile is read in the input's
// contiguous order and written in the output's, so both sides are coalesced.
constexpr int kTpSites = 32, kTpCols = 8;

template <typename Ti, typename To>
__global__ __launch_bounds__(256) void transpose_kernel(int64_t V, int cols, const cx<Ti> *__restrict__ in,
                                                        Strides si, int in_cm, cx<To> *__restrict__ out,
                                                        Strides so, int accumulate, double scale) {
    // [site][comp][col], one padding element per site against bank conflicts
    constexpr int kSiteStride = 12 * kTpCols + 1;
    __shared__ cx<double> tile[kTpSites * kSiteStride];
    const int64_t x0 = (int64_t)blockIdx.x * kTpSites;
    const int ns = (int)min((int64_t)kTpSites, V - x0);
    for (int r0 = 0; r0 < cols; r0 += kTpCols) {
        const int nc = min(kTpCols, cols - r0);
        const int nel = ns * 12 * nc;
        __syncthreads();
        for (int e = threadIdx.x; e < nel; e += blockDim.x) {
            int x, c, r;
            if (in_cm) {  // sites fastest
                x = e % ns;
                const int k = e / ns;
                c = k % 12;
                r = k / 12;
            } else {      // columns fastest
                r = e % nc;
                const int k = e / nc;
                c = k % 12;
                x = k / 12;
            }
            const cx<double> v = cvt<double>(in[si.base + (x0 + x) * si.site + c * si.comp + (r0 + r) * si.col]);
            tile[x * kSiteStride + c * kTpCols + r] = mk<double>(scale * v.x, scale * v.y);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nel; e += blockDim.x) {
            int x, c, r;
            if (in_cm) {  // output [V][12][ld]: columns fastest
                r = e % nc;
                const int k = e / nc;
                c = k % 12;
                x = k / 12;
            } else {      // output column-major: sites fastest
                x = e % ns;
                const int k = e / ns;
                c = k % 12;
                r = k / 12;
            }
            const cx<double> v = tile[x * kSiteStride + c * kTpCols + r];
            cx<To> *o = out + so.base + (x0 + x) * so.site + c * so.comp + (r0 + r) * so.col;
            if (accumulate) {
                const cx<double> w = cvt<double>(*o);
                *o = cvt<To>(mk<double>(w.x + v.x, w.y + v.y));
            } else {
                *o = cvt<To>(v);
            }
        }
    }
}

hipError_t copy_field(int64_t V, int cols, FieldDesc in, FieldDesc out, bool accumulate,
                      double scale, hipStream_t st) {
    if (in.layout != out.layout) {
        const Strides si = strides_of(in, V), so = strides_of(out, V);
        const dim3 grid((unsigned)((V + kTpSites - 1) / kTpSites));
        const int icm = in.layout == kCM, acc = accumulate ? 1 : 0;
#define DSBCG_TP(TI, TO)                                                                       \
    hipLaunchKernelGGL((transpose_kernel<TI, TO>), grid, dim3(256), 0, st, V, cols,            \
                       (const cx<TI> *)in.p, si, icm, (cx<TO> *)out.p, so, acc, scale)
        if (in.fp64 && out.fp64)
            DSBCG_TP(double, double);
        else if (in.fp64)
            DSBCG_TP(double, float);
        else if (out.fp64)
            DSBCG_TP(float, double);
        else
            DSBCG_TP(float, float);
#undef DSBCG_TP
        return hipGetLastError();
    }
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
// Window update on the matrix cores.  For shift j the window contraction is
//   [out_X | out_P] (rows x (m + bend)) = [P_{j,i0} | V_window] (rows x K_in) * C_j
// in complex arithmetic.  It runs as a real product with 16x16x4 MFMAs in the
// transposed orientation: the A operand is the coefficient table (output
// real columns x 4 input reals = one pair of complex inputs), the B operand
// is the data (4 input reals x 16 rows).  The table orders the output reals
// so that lane group g = lane / 16 ends with (re, im) of the complex
// outputs 8 mt + 2 g and 8 mt + 2 g + 1 of one data row in its four
// accumulators; each lane group then stores 16 consecutive rows.
//
// A workgroup owns 16 * TILES consecutive rows and has one wave per shift of
// the window; the window columns are staged chunk by chunk in LDS (double
// buffered, asynchronous copies) and read by every wave, the P_{j,i0}
// columns are read by their own wave only.
// ---------------------------------------------------------------------------
template <typename R>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 mac(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 mac(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// Stage geometry of the window contraction: PAIRS input pairs (2 PAIRS
// columns) of the workgroup's 64 rows, plus the coefficients of those pairs
// for every shift of the launch.  Fewer pairs for wide outputs.
template <typename R, int NMT>
struct WinStage {
    static constexpr int pairs = NMT == 1 ? 4 : (NMT == 2 ? 2 : 1);
    static constexpr int rows = 64;                                  // rows per workgroup
    static constexpr int rpl = 16 / (int)sizeof(cx<R>);              // rows per lane and copy
    static constexpr int data_bytes = 2 * pairs * rows * (int)sizeof(cx<R>);
    static constexpr int data_copies = data_bytes / 1024;            // 1 KiB copies
    static constexpr int coef_elems = pairs * NMT * 64;               // per shift
    static constexpr int coef_bytes = coef_elems * (int)sizeof(R);
    static constexpr int coef_copies = (coef_bytes + 1023) / 1024;
    static_assert(data_bytes % 1024 == 0 && coef_bytes % 16 == 0, "16-byte lanes, 1 KiB copies");
};

// Issue the asynchronous global-to-LDS copies of stage k into buf: the data
// block [column][64 rows] of cx<R>, then per shift the table entries
// [pair][mt][lane] of the stage's pairs.  Lane l of a copy writes 16 bytes
// at (copy base) + 16 l; the waves share the copies.  Columns past the
// window, rows past n and pairs past the table read column 0 / row 0 /
// pair 0 instead: they are skipped or their outputs discarded, so only
// finite values matter there.  FP32 rows move in aligned pairs (n even).
template <typename R, int NMT>
__device__ inline void stage_window(const WinArgs &a, int k, int64_t r0, char *buf, int lane, int wave,
                                    int nw) {
    typedef WinStage<R, NMT> S;
    const int npairs_v = (a.ncolv + 1) >> 1;
    const int total = S::data_copies + a.nshift * S::coef_copies;
    for (int q = wave; q < total; q += nw) {
        const void *src;
        char *dst;
        if (q < S::data_copies) {
            const int e = q * 64 * S::rpl + lane * S::rpl;
            const int cc = e / S::rows, r = e - cc * S::rows;
            const int c = k * 2 * S::pairs + cc;
            int64_t row = r0 + r;
            if (row >= a.nrows) row = 0;
            src = (const cx<R> *)a.colptr[c < a.ncolv ? c : 0] + row;
            dst = buf + q * 1024;
        } else {
            const int js = (q - S::data_copies) / S::coef_copies;
            const int cq = (q - S::data_copies) - js * S::coef_copies;
            const int byte = cq * 1024 + lane * 16;
            if (byte >= S::coef_bytes) continue;  // partial last copy
            const int e = byte / (int)sizeof(R);
            int pair = k * S::pairs + e / (NMT * 64);
            const int rest = e % (NMT * 64);
            if (pair >= npairs_v) pair = 0;
            src = (const R *)a.table + ((size_t)js * a.npairs + a.pairs_p + pair) * NMT * 64 + rest;
            dst = buf + S::data_bytes + js * S::coef_bytes + cq * 1024;
        }
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
    }
}

// The staged window columns of one precision (a.colptr, a.ncolv, a.table),
// multiplied into acc.  With issued, stage 0 is already on its way into the
// first buffer; otherwise it is issued here once every wave is done with
// the buffers.
template <typename R, int NMT, int SPW>
__device__ inline void window_stages(const WinArgs &a, char *smem, int64_t r0, int lane, int wave, int nw,
                                     int tile, int js0, int nsw, bool issued,
                                     typename Mfma<R>::v4 (&acc)[SPW][NMT]) {
    typedef WinStage<R, NMT> S;
    const int rl = lane & 15, part = (lane >> 4) & 1, sel = lane >> 5;
    const int npairs_v = (a.ncolv + 1) >> 1;
    const int nst = (npairs_v + S::pairs - 1) / S::pairs;
    const int buf_bytes = S::data_bytes + a.nshift * S::coef_bytes;
    if (!issued) {
        __syncthreads();
        if (nst > 0) stage_window<R, NMT>(a, 0, r0, smem, lane, wave, nw);
    }
    for (int k = 0; k < nst; ++k) {
        // stage k has landed for every wave, and every wave is done with
        // stage k - 1, whose buffer takes stage k + 1
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (k + 1 < nst) stage_window<R, NMT>(a, k + 1, r0, smem + ((k + 1) & 1) * buf_bytes, lane, wave, nw);
        const char *buf = smem + (k & 1) * buf_bytes;
        const cx<R> *dat = (const cx<R> *)buf;
        const R *cof = (const R *)(buf + S::data_bytes) + (size_t)js0 * S::coef_elems + lane;
        const int npp = min(S::pairs, npairs_v - k * S::pairs);
#pragma unroll
        for (int pp = 0; pp < S::pairs; ++pp) {
            if (pp < npp) {
                const R d = ((const R *)&dat[(2 * pp + sel) * S::rows + tile * 16 + rl])[part];
#pragma unroll
                for (int u = 0; u < SPW; ++u) {
                    if (u < nsw) {
#pragma unroll
                        for (int mt = 0; mt < NMT; ++mt)
                            acc[u][mt] = Mfma<R>::mac(cof[u * S::coef_elems + (pp * NMT + mt) * 64], d, acc[u][mt]);
                    }
                }
            }
        }
    }
}

// Workgroup: 64 rows, 4 waves per group of up to SPW shifts; wave w takes the
// 16-row tile w % 4 for the shifts of group w / 4.  Each SIMD thus holds one
// wave of every group and the matrix-core work is the same on all four.
// The stages are double buffered: the copies of stage k + 1 run while stage
// k multiplies; every operand of the multiply comes from LDS.  TWO: a second
// part of the window in FP32 (see WinArgs).
template <typename R, int NMT, int SPW, bool TWO>
__global__ __launch_bounds__(1024) void window_kernel(WinArgs a) {
    typedef WinStage<R, NMT> S;
    typedef typename Mfma<R>::v4 v4;
    typedef typename Mfma<float>::v4 v4f;
    extern __shared__ __align__(16) char win_smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int grp = wave >> 2, tile = wave & 3;
    const int64_t n = a.nrows;
    const int64_t r0 = (int64_t)blockIdx.x * S::rows;
    const int rl = lane & 15;           // row within the tile
    const int part = (lane >> 4) & 1;   // real (0) or imaginary (1) part of the input
    const int sel = lane >> 5;          // input column of the pair
    const int64_t row = r0 + tile * 16 + rl;
    const int js0 = grp * SPW;
    const int nsw = min(SPW, a.nshift - js0);  // >= 1 by the launch shape

    // the first stage's copies overlap the P_{j,i0} part
    if (a.ncolv > 0) stage_window<R, NMT>(a, 0, r0, win_smem, lane, wave, nw);

    v4 acc[SPW][NMT];
    v4f acc2[SPW][NMT];
#pragma unroll
    for (int u = 0; u < SPW; ++u)
#pragma unroll
        for (int mt = 0; mt < NMT; ++mt) {
            acc[u][mt] = v4{0, 0, 0, 0};
            acc2[u][mt] = v4f{0, 0, 0, 0};
        }

    // inputs from P_{j,i0}, per shift; coefficients straight from the table
    if (a.bp0 > 0) {
#pragma unroll
        for (int u = 0; u < SPW; ++u) {
            if (u >= nsw) break;
            const int js = js0 + u;
            const R *P = (const R *)a.Pold + (size_t)2 * a.shifts[js] * a.pstride;
            const R *tab = (const R *)a.table + (size_t)js * a.npairs * NMT * 64 + lane;
            for (int pp = 0; pp < a.pairs_p; ++pp) {
                const int p = 2 * pp + sel;
                const R d = (p < a.bp0 && row < n) ? P[2 * ((int64_t)p * n + row) + part] : (R)0;
#pragma unroll
                for (int mt = 0; mt < NMT; ++mt)
                    acc[u][mt] = Mfma<R>::mac(tab[(pp * NMT + mt) * 64], d, acc[u][mt]);
            }
        }
    }
    window_stages<R, NMT, SPW>(a, win_smem, r0, lane, wave, nw, tile, js0, nsw, true, acc);
    if (TWO) {
        // the FP32 part of the window, in the same buffers
        WinArgs b = a;
        b.ncolv = a.ncolv2;
        b.colptr = a.colptr2;
        b.table = a.table2;
        b.npairs = a.npairs2;
        b.pairs_p = 0;
        b.bp0 = 0;
        window_stages<float, NMT, SPW>(b, win_smem, r0, lane, wave, nw, tile, js0, nsw, false, acc2);
    }
    if (row >= n) return;
    // lane holds row `row`, complex outputs q = 8 mt + 2 g and q + 1 of each shift
    const int g = lane >> 4;
    // row = c V + x (spin-colour c, site x) is element (x, c) of the caller's layout
    const int64_t Vs = n / 12, cs = row / Vs;
    const int64_t api_row = ((row - cs * Vs) * 12 + cs) * a.m;
#pragma unroll
    for (int u = 0; u < SPW; ++u) {
        if (u >= nsw) break;
        const int j = a.shifts[js0 + u];
        const uint32_t xm = a.xmask[j];
        const bool wp = a.pmask[j] != 0;
        zd *X = a.X + (size_t)j * a.xstride;
#pragma unroll
        for (int mt = 0; mt < NMT; ++mt) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = mt * 8 + 2 * g + h;
                double re = (double)acc[u][mt][2 * h], im = (double)acc[u][mt][2 * h + 1];
                if (TWO) {
                    re += (double)acc2[u][mt][2 * h];
                    im += (double)acc2[u][mt][2 * h + 1];
                }
                if (q < a.m) {
                    zd *x = X + (int64_t)q * n + row;
                    // first window: X_j = increment (zero where never updated)
                    if (a.xinit || ((xm >> q) & 1u)) {
                        const zd v = a.xinit ? mk<double>(re, im) : mk<double>(x->x + re, x->y + im);
                        *x = v;
                        if (a.Xapi) a.Xapi[(int64_t)j * n * a.m + api_row + q] = v;
                    } else if (a.Xapi) {
                        a.Xapi[(int64_t)j * n * a.m + api_row + q] = *x;
                    }
                } else if (wp && q - a.m < a.bend) {
                    const int64_t at = (int64_t)j * a.pstride + (int64_t)(q - a.m) * n + row;
                    if (TWO)
                        ((zf *)a.Pnew2)[at] = mk<float>((float)re, (float)im);
                    else
                        ((cx<R> *)a.Pnew)[at] = mk<R>((R)re, (R)im);
                }
            }
        }
    }
}

template <typename R, int NMT, int SPW>
hipError_t window_launch(const WinArgs &a, hipStream_t st) {
    typedef WinStage<R, NMT> S;
    const int groups = (a.nshift + SPW - 1) / SPW;
    const dim3 block(64 * 4 * groups);
    const dim3 grid((unsigned)((a.nrows + S::rows - 1) / S::rows));
    const size_t lds = 2 * ((size_t)S::data_bytes + (size_t)a.nshift * S::coef_bytes);
    if constexpr (sizeof(R) == 8) {
        if (a.ncolv2 > 0) {
            hipLaunchKernelGGL((window_kernel<R, NMT, SPW, true>), grid, block, lds, st, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((window_kernel<R, NMT, SPW, false>), grid, block, lds, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Three-product form of the window contraction.  For c = a + ib, the
// coefficient of input d = dr + i di in one output, the real 2 x 2 form
// above spends four real products; here three real contractions over the
// window's complex inputs give
//   T1 = sum a dr,  T2 = sum b di,  T3 = sum (a + b)(dr + di),
//   Re out = T1 - T2,  Im out = T3 - T1 - T2,
// a quarter fewer matrix-core products and table entries.  The A operand
// (16 rows x 4 inputs) holds the 8 outputs of each of two shifts, which
// share the B operand (4 complex inputs x 16 rows, one real combination per
// contraction); the lane order of small_window_table3 puts output
// 2 g + (r & 1) of shift 2 js2 + (r >> 1) in register r of lane group g in
// both precisions.  Stages of 8 window columns (two blocks of 4) and the
// tables of all shift pairs of the launch are double buffered in LDS as in
// window_kernel.  The FP32 part of a window across the switch runs in
// window_kernel's real 2 x 2 form, whose two accumulators per output leave
// room for the FP64 part's results.  Used for windows with no P_{j,i0}
// inputs and at most 8 outputs per shift; the others take window_kernel.
// ---------------------------------------------------------------------------
template <typename R>
struct Win3Stage {
    static constexpr int blocks = 2;                                  // blocks of 4 columns
    static constexpr int rows = 64;                                   // rows per workgroup
    static constexpr int rpl = 16 / (int)sizeof(cx<R>);               // rows per lane and copy
    static constexpr int data_bytes = 4 * blocks * rows * (int)sizeof(cx<R>);
    static constexpr int data_copies = data_bytes / 1024;
    static constexpr int coef_elems = blocks * 3 * 64;                // per shift pair
    static constexpr int coef_bytes = coef_elems * (int)sizeof(R);
    static constexpr int coef_copies = (coef_bytes + 1023) / 1024;
    static_assert(data_bytes % 1024 == 0 && coef_bytes % 16 == 0, "16-byte lanes, 1 KiB copies");
};

// Asynchronous copies of stage k into buf: the data block [column][64 rows],
// then per shift pair the table entries [block][t][lane] of the stage's
// blocks.  Columns past the window, rows past n and blocks past the table
// read column 0 / row 0 / block 0 (finite values whose products are
// discarded or multiplied by zero coefficients).
template <typename R>
__device__ inline void stage_window3(const WinArgs &a, int k, int64_t r0, char *buf, int lane, int wave,
                                     int nw) {
    typedef Win3Stage<R> S;
    const int nblk = (a.ncolv + 3) >> 2, np2 = (a.nshift + 1) >> 1;
    const int total = S::data_copies + np2 * S::coef_copies;
    for (int q = wave; q < total; q += nw) {
        const void *src;
        char *dst;
        if (q < S::data_copies) {
            const int e = q * 64 * S::rpl + lane * S::rpl;
            const int cc = e / S::rows, r = e - cc * S::rows;
            const int c = k * 4 * S::blocks + cc;
            int64_t row = r0 + r;
            if (row >= a.nrows) row = 0;
            src = (const cx<R> *)a.colptr[c < a.ncolv ? c : 0] + row;
            dst = buf + q * 1024;
        } else {
            const int jp = (q - S::data_copies) / S::coef_copies;
            const int cq = (q - S::data_copies) - jp * S::coef_copies;
            const int byte = cq * 1024 + lane * 16;
            if (byte >= S::coef_bytes) continue;  // partial last copy
            const int e = byte / (int)sizeof(R);
            int blk = k * S::blocks + e / (3 * 64);
            const int rest = e % (3 * 64);
            if (blk >= nblk) blk = 0;
            src = (const R *)a.table + ((size_t)jp * nblk + blk) * 3 * 64 + rest;
            dst = buf + S::data_bytes + jp * S::coef_bytes + cq * 1024;
        }
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
    }
}

template <typename R, int SPW2>
__device__ inline void window3_stages(const WinArgs &a, char *smem, int64_t r0, int lane, int wave, int nw,
                                      int tile, int jp0, int npw, bool issued,
                                      typename Mfma<R>::v4 (&acc)[SPW2][3]) {
    typedef Win3Stage<R> S;
    const int rl = lane & 15, kk = lane >> 4;
    const int nblk = (a.ncolv + 3) >> 2, np2 = (a.nshift + 1) >> 1;
    const int nst = (nblk + S::blocks - 1) / S::blocks;
    const int buf_bytes = S::data_bytes + np2 * S::coef_bytes;
    if (!issued) {
        __syncthreads();
        if (nst > 0) stage_window3<R>(a, 0, r0, smem, lane, wave, nw);
    }
    for (int k = 0; k < nst; ++k) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (k + 1 < nst) stage_window3<R>(a, k + 1, r0, smem + ((k + 1) & 1) * buf_bytes, lane, wave, nw);
        const char *buf = smem + (k & 1) * buf_bytes;
        const cx<R> *dat = (const cx<R> *)buf;
        const R *cof = (const R *)(buf + S::data_bytes) + (size_t)jp0 * S::coef_elems + lane;
        const int nb = min(S::blocks, nblk - k * S::blocks);
#pragma unroll
        for (int bb = 0; bb < S::blocks; ++bb) {
            if (bb < nb) {
                const cx<R> d = dat[(4 * bb + kk) * S::rows + tile * 16 + rl];
                const R dr = d.x, di = d.y, ds = d.x + d.y;
#pragma unroll
                for (int u = 0; u < SPW2; ++u) {
                    if (u < npw) {
                        const R *cu = cof + u * S::coef_elems + bb * 3 * 64;
                        acc[u][0] = Mfma<R>::mac(cu[0], dr, acc[u][0]);
                        acc[u][1] = Mfma<R>::mac(cu[64], di, acc[u][1]);
                        acc[u][2] = Mfma<R>::mac(cu[128], ds, acc[u][2]);
                    }
                }
            }
        }
    }
}

// Workgroup: 64 rows, 4 waves per group of up to SPW2 shift pairs; wave w
// takes the 16-row tile w % 4 for the pairs of group w / 4.  TWO: the FP32
// part of a window across the switch (see WinArgs), added in FP64.
template <typename R, int SPW2, bool TWO>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6))) void window3_kernel(WinArgs a) {
    typedef typename Mfma<R>::v4 v4;
    typedef typename Mfma<float>::v4 v4f;
    extern __shared__ __align__(16) char win3_smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int grp = wave >> 2, tile = wave & 3;
    const int64_t n = a.nrows;
    const int64_t r0 = (int64_t)blockIdx.x * Win3Stage<R>::rows;
    const int64_t row = r0 + tile * 16 + (lane & 15);
    const int np2 = (a.nshift + 1) >> 1;
    const int jp0 = grp * SPW2;
    const int npw = min(SPW2, np2 - jp0);  // >= 1 by the launch shape

    if (a.ncolv > 0) stage_window3<R>(a, 0, r0, win3_smem, lane, wave, nw);
    v4 acc[SPW2][3];
#pragma unroll
    for (int u = 0; u < SPW2; ++u)
#pragma unroll
        for (int t = 0; t < 3; ++t) acc[u][t] = v4{0, 0, 0, 0};
    window3_stages<R, SPW2>(a, win3_smem, r0, lane, wave, nw, tile, jp0, npw, true, acc);
    // the first part's outputs as (re, im) while the FP32 part runs: two
    // registers per output instead of three
    double ore[SPW2][4], oim[SPW2][4];
#pragma unroll
    for (int u = 0; u < SPW2; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double t1 = (double)acc[u][0][r], t2 = (double)acc[u][1][r], t3 = (double)acc[u][2][r];
            ore[u][r] = t1 - t2;
            oim[u][r] = t3 - t1 - t2;
            if (TWO) {
                // formed here, not after the FP32 part (which would keep
                // the three sums alive through it)
                __asm__ volatile("" : "+v"(ore[u][r]), "+v"(oim[u][r]));
            }
        }
    if (TWO) {
        // the FP32 part in the real 2 x 2 form of window_kernel (table2 from
        // small_window_table): two accumulators per output instead of three
        // keep the first part's outputs in registers
        WinArgs b = a;
        b.ncolv = a.ncolv2;
        b.colptr = a.colptr2;
        b.table = a.table2;
        b.npairs = a.npairs2;
        b.pairs_p = 0;
        b.bp0 = 0;
        v4f acc2[2 * SPW2][1];
#pragma unroll
        for (int u = 0; u < 2 * SPW2; ++u) acc2[u][0] = v4f{0, 0, 0, 0};
        const int js0 = 2 * jp0, nsw = min(2 * SPW2, a.nshift - js0);
        window_stages<float, 1, 2 * SPW2>(b, win3_smem, r0, lane, wave, nw, tile, js0, nsw, false, acc2);
        // shift 2 u + (r >> 1) of the wave, output 2 g + (r & 1): (re, im) in
        // registers 2 (r & 1), 2 (r & 1) + 1 of its accumulator
#pragma unroll
        for (int u = 0; u < SPW2; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ore[u][r] += (double)acc2[2 * u + (r >> 1)][0][2 * (r & 1)];
                oim[u][r] += (double)acc2[2 * u + (r >> 1)][0][2 * (r & 1) + 1];
            }
    }
    if (row >= n) return;
    const int g = lane >> 4;
    const int64_t Vs = n / 12, cs = row / Vs;
    const int64_t api_row = ((row - cs * Vs) * 12 + cs) * a.m;
#pragma unroll
    for (int u = 0; u < SPW2; ++u) {
        if (u >= npw) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int js = 2 * (jp0 + u) + (r >> 1), q = 2 * g + (r & 1);
            if (js >= a.nshift) continue;
            const double re = ore[u][r], im = oim[u][r];
            const int j = a.shifts[js];
            if (q < a.m) {
                zd *x = a.X + (size_t)j * a.xstride + (int64_t)q * n + row;
                if (a.xinit || ((a.xmask[j] >> q) & 1u)) {
                    const zd v = a.xinit ? mk<double>(re, im) : mk<double>(x->x + re, x->y + im);
                    *x = v;
                    if (a.Xapi) a.Xapi[(int64_t)j * n * a.m + api_row + q] = v;
                } else if (a.Xapi) {
                    a.Xapi[(int64_t)j * n * a.m + api_row + q] = *x;
                }
            } else if (a.pmask[j] != 0 && q - a.m < a.bend) {
                const int64_t at = (int64_t)j * a.pstride + (int64_t)(q - a.m) * n + row;
                if (TWO)
                    ((zf *)a.Pnew2)[at] = mk<float>((float)re, (float)im);
                else
                    ((cx<R> *)a.Pnew)[at] = mk<R>((R)re, (R)im);
            }
        }
    }
}

template <typename R, int SPW2>
hipError_t window3_launch(const WinArgs &a, hipStream_t st) {
    typedef Win3Stage<R> S;
    const int np2 = (a.nshift + 1) / 2;
    const int groups = (np2 + SPW2 - 1) / SPW2;
    const dim3 block(64 * 4 * groups);
    const dim3 grid((unsigned)((a.nrows + S::rows - 1) / S::rows));
    const size_t lds = 2 * ((size_t)S::data_bytes + (size_t)np2 * S::coef_bytes);
    if constexpr (sizeof(R) == 8) {
        if (a.ncolv2 > 0) {
            hipLaunchKernelGGL((window3_kernel<R, SPW2, true>), grid, block, lds, st, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((window3_kernel<R, SPW2, false>), grid, block, lds, st, a);
    return hipGetLastError();
}

template <typename R, int NMT>
hipError_t window_launch_spw(const WinArgs &a, int spw, hipStream_t st) {
    if (spw == 1) return window_launch<R, NMT, 1>(a, st);
    // wide FP64 outputs keep at most two shifts' accumulators per wave
    if constexpr (sizeof(R) == 8 && NMT >= 3) {
        return window_launch<R, NMT, 2>(a, st);
    } else {
        if (spw == 2) return window_launch<R, NMT, 2>(a, st);
        return window_launch<R, NMT, 4>(a, st);
    }
}

hipError_t window_apply(bool fp64, const WinArgs &a, hipStream_t st) {
    // m = 0: only P_{j,end} is formed (partial-fraction form).  The staged
    // copies move rows in aligned pairs in FP32: nrows must be even.
    if (a.nshift < 1 || a.nshift > 16 || a.m < 0 || a.m > 16 || a.bend < 0 || a.bend > 16 ||
        (a.nrows & 1) || (a.ncolv > 0 && !a.colptr) ||
        a.m + a.bend < 1 || (a.m == 0 && a.xinit) ||
        a.bp0 < 0 || a.bp0 > 16 || a.ncolv < 0 || a.nmt < 1 || a.nmt > 4 ||
        a.nmt * 8 < a.m + a.bend || a.pairs_p != (a.bp0 + 1) / 2 ||
        a.npairs != a.pairs_p + (a.ncolv + 1) / 2 ||
        (a.ncolv2 > 0 && (!fp64 || !a.colptr2 || !a.table2 || a.npairs2 != (a.ncolv2 + 1) / 2 ||
                          (a.bend > 0 && !a.Pnew2))) ||
        (a.Xapi && (a.nrows % 12 != 0 || a.m < 1)))
        return hipErrorInvalidValue;
    if (a.nrows <= 0) return hipSuccess;
    if (a.gauss) {
        // all shift pairs in one launch: at most 4 groups of 2 pairs, and
        // 2 (8 KiB + 8 x 3 KiB) of LDS in FP64
        if (a.bp0 != 0 || a.nmt != 1 || a.m + a.bend > 8 || (a.ncolv2 > 0 && a.table2 == nullptr))
            return hipErrorInvalidValue;
        const int np2 = (a.nshift + 1) / 2;
        if (fp64) return np2 <= 4 ? window3_launch<double, 1>(a, st) : window3_launch<double, 2>(a, st);
        return np2 <= 4 ? window3_launch<float, 1>(a, st) : window3_launch<float, 2>(a, st);
    }
    // shifts per launch: at most 16 waves (4 groups) of SPW <= 4 shifts, FP64
    // accumulators of wide outputs in at most 2 shifts per wave, and at most
    // 64 KiB of double-buffered LDS
    const size_t esz = fp64 ? sizeof(double) : sizeof(float);
    const int max_spw = (fp64 && a.nmt >= 3) ? 2 : 4;
    const int pairs = a.nmt == 1 ? 4 : (a.nmt == 2 ? 2 : 1);
    const size_t data_bytes = 2 * (size_t)pairs * 64 * 2 * esz, coef_bytes = (size_t)pairs * a.nmt * 64 * esz;
    const int lds_cnt = (int)((32768 - data_bytes) / coef_bytes);
    const int max_cnt = std::min(std::min(16, 4 * max_spw), lds_cnt);
    for (int js0 = 0; js0 < a.nshift; js0 += max_cnt) {
        WinArgs b = a;
        b.nshift = std::min(max_cnt, a.nshift - js0);
        b.shifts = a.shifts + js0;
        b.table = (const char *)a.table + (size_t)js0 * a.npairs * a.nmt * 64 * esz;
        if (a.ncolv2 > 0) b.table2 = (const char *)a.table2 + (size_t)js0 * a.npairs2 * a.nmt * 64 * sizeof(float);
        const int spw = b.nshift <= 4 ? 1 : (b.nshift <= 8 ? 2 : 4);
        hipError_t e;
#define DSBCG_WIN(R)                                                        \
    switch (a.nmt) {                                                        \
    case 1: e = window_launch_spw<R, 1>(b, spw, st); break;                 \
    case 2: e = window_launch_spw<R, 2>(b, spw, st); break;                 \
    case 3: e = window_launch_spw<R, 3>(b, spw, st); break;                 \
    default: e = window_launch_spw<R, 4>(b, spw, st); break;                \
    }
        if (fp64) {
            DSBCG_WIN(double)
        } else {
            DSBCG_WIN(float)
        }
#undef DSBCG_WIN
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Partial-fraction window update (see RatArgs).  Lane layout as in
// window_kernel: lane = row + 16 k, k = 2 (input column of the pair) +
// (real / imaginary part); the next pair's inputs and coefficients are
// loaded while the current pair multiplies.
template <typename R, int NMT, int TILES>
__global__ __launch_bounds__(256) void rational_window_kernel(RatArgs a) {
    typedef typename Mfma<R>::v4 v4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t n = a.nrows;
    const int64_t r0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * 16 * TILES;
    if (r0 >= n) return;  // no barriers below: a wave past the end just leaves
    const int rl = lane & 15, part = (lane >> 4) & 1, sel = lane >> 5;
    const R *tab = (const R *)a.table + lane;
    const int npp = a.nshift * a.pairs_p;  // pairs from the P_{j,i0}
    const int npairs = a.npairs;

    // input (pair, tile) of this lane: P_{j,i0} pairs first, then window columns
    auto load = [&](int pair, R d[TILES]) {
        const R *src = nullptr;
        int64_t off = 0;
        if (pair < npp) {
            const int js = pair / a.pairs_p, p = 2 * (pair - js * a.pairs_p) + sel;
            if (p < a.bp0) {
                src = (const R *)a.Pold + (size_t)2 * a.shifts[js] * a.pstride;
                off = 2 * (int64_t)p * n;
            }
        } else {
            const int col = 2 * (pair - npp) + sel;
            if (col < a.ncolv) src = (const R *)a.colptr[col];
        }
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
            const int64_t row = r0 + t * 16 + rl;
            d[t] = (src && row < n) ? src[off + 2 * row + part] : (R)0;
        }
    };

    v4 acc[TILES][NMT];
#pragma unroll
    for (int t = 0; t < TILES; ++t)
#pragma unroll
        for (int mt = 0; mt < NMT; ++mt) acc[t][mt] = v4{0, 0, 0, 0};
    R d[TILES], cf[NMT];
    load(0, d);
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt) cf[mt] = tab[mt * 64];
    for (int pr = 0; pr < npairs; ++pr) {
        const int pn = pr + 1 < npairs ? pr + 1 : pr;
        R dn[TILES], cn[NMT];
        load(pn, dn);
#pragma unroll
        for (int mt = 0; mt < NMT; ++mt) cn[mt] = tab[((size_t)pn * NMT + mt) * 64];
#pragma unroll
        for (int mt = 0; mt < NMT; ++mt)
#pragma unroll
            for (int t = 0; t < TILES; ++t) acc[t][mt] = Mfma<R>::mac(cf[mt], d[t], acc[t][mt]);
#pragma unroll
        for (int t = 0; t < TILES; ++t) d[t] = dn[t];
#pragma unroll
        for (int mt = 0; mt < NMT; ++mt) cf[mt] = cn[mt];
    }
    // lane holds rows r0 + 16 t + rl, complex outputs q = 8 mt + 2 g and q + 1
    const int g = lane >> 4;
#pragma unroll
    for (int t = 0; t < TILES; ++t) {
        const int64_t row = r0 + t * 16 + rl;
        if (row >= n) continue;
#pragma unroll
        for (int mt = 0; mt < NMT; ++mt)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = mt * 8 + 2 * g + h;
                if (q < a.m) {
                    zd *y = a.Y + (int64_t)q * n + row;
                    *y = mk<double>(y->x + (double)acc[t][mt][2 * h], y->y + (double)acc[t][mt][2 * h + 1]);
                }
            }
    }
}

hipError_t rational_window_apply(bool fp64, const RatArgs &a, hipStream_t st) {
    if (a.nshift < 1 || a.nshift > 16 || a.m < 1 || a.m > 16 || a.bp0 < 0 || a.bp0 > 16 ||
        a.ncolv < 0 || a.pairs_p != (a.bp0 + 1) / 2 || a.nmt != (a.m + 7) / 8 ||
        a.npairs != a.nshift * a.pairs_p + (a.ncolv + 1) / 2 || !a.Y || !a.table)
        return hipErrorInvalidValue;
    if (a.nrows <= 0 || a.npairs == 0) return hipSuccess;
    constexpr int kWaves = 4;
    const int tiles = fp64 ? 4 : 8;
    const int64_t rows_per_wg = (int64_t)kWaves * 16 * tiles;
    const dim3 grid((unsigned)((a.nrows + rows_per_wg - 1) / rows_per_wg)), block(64 * kWaves);
#define DSBCG_RW(R, M, T) hipLaunchKernelGGL((rational_window_kernel<R, M, T>), grid, block, 0, st, a)
    if (fp64) {
        if (a.nmt == 1) DSBCG_RW(double, 1, 4);
        else DSBCG_RW(double, 2, 4);
    } else {
        if (a.nmt == 1) DSBCG_RW(float, 1, 8);
        else DSBCG_RW(float, 2, 8);
    }
#undef DSBCG_RW
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
