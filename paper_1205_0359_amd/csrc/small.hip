// Small FP64 algebra of DSBlockCG, on the device.
//
// Block form of the paper's root-free Cholesky recurrences (Sec. 3): for
// T_sigma = sigma I + T, block tridiagonal with diagonal blocks alpha_i and
// sub-diagonal blocks beta_{i+1},
//   Delta_{j,1} = alpha_1 + sigma_j I
//   N_{j,i}     = Delta_{j,i-1}^{-1} beta_i^H
//   Delta_{j,i} = alpha_i + sigma_j I - beta_i N_{j,i}
//   M_{j,i}     = Delta_{j,i}^{-1} Z_{j,i}
//   Z_{j,i+1}   = -beta_{i+1} M_{j,i}  (the residual coefficients: R_j = V_{i+1} Z_{j,i+1})
// with Z_{j,1} = rho from B = V_1 rho.  The block Lanczos basis is made
// orthonormal by a deflated Cholesky QR applied twice.
//
// These matrices are at most 16 x 16; each kernel runs one or a few
// workgroups.

#include "small.hpp"

namespace dsbcg {

__device__ inline zd zmul(zd a, zd b) { return a * b; }
__device__ inline zd zdivr(zd a, double r) { return mk<double>(a.x / r, a.y / r); }

// Forward substitution L y = y (L lower, n x n, leading dim 16) on one column
// held by this thread; stride gives the column's element spacing.
__device__ inline void lower_solve(const zd *L, zd *y, int n, int stride) {
    for (int r = 0; r < n; ++r) {
        zd v = y[r * stride];
        for (int c = 0; c < r; ++c) {
            const zd l = L[r * 16 + c];
            const zd w = y[c * stride];
            v = v - l * w;
        }
        y[r * stride] = zdivr(v, L[r * 16 + r].x);
    }
}

// Back substitution L^H y = y.
__device__ inline void lower_h_solve(const zd *L, zd *y, int n, int stride) {
    for (int r = n - 1; r >= 0; --r) {
        zd v = y[r * stride];
        for (int c = r + 1; c < n; ++c) {
            const zd l = conj(L[c * 16 + r]);
            v = v - l * y[c * stride];
        }
        y[r * stride] = zdivr(v, L[r * 16 + r].x);
    }
}

// ---------------------------------------------------------------------------
// Per-shift coefficients: one 64-lane workgroup per active shift.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void shift_coeffs_kernel(SmallState *st, StepReport *rep,
                                                          const zd *__restrict__ alpha_raw,
                                                          int first,
                                                          const int32_t *__restrict__ list) {
    __shared__ zd A[256], Bt[256], Lp[256], Nn[256], D[256], Zs[256];
    const int j = list[blockIdx.x];
    const int t = threadIdx.x;
    const int b = st->b, bp = st->bp, m = st->m;
    const double sg = st->sigma[j];

    (void)alpha_raw;
    for (int e = t; e < b * b; e += 64) {
        const int r = e / b, c = e - r * b;
        A[r * 16 + c] = st->alpha[r * 16 + c];
    }
    if (!first) {
        for (int e = t; e < b * bp; e += 64) {
            const int r = e / bp, c = e - r * bp;
            Bt[r * 16 + c] = st->beta[r * 16 + c];
        }
        for (int e = t; e < bp * bp; e += 64) {
            const int r = e / bp, c = e - r * bp;
            Lp[r * 16 + c] = st->L[j][r * 16 + c];
        }
    }
    __syncthreads();

    if (first) {
        for (int e = t; e < b * b; e += 64) {
            const int r = e / b, c = e - r * b;
            zd v = A[r * 16 + c];
            if (r == c) v.x += sg;
            D[r * 16 + c] = v;
        }
    } else {
        // N = Delta_{i-1}^{-1} beta^H: column q of beta^H per lane
        if (t < b) {
            for (int p = 0; p < bp; ++p) Nn[p * 16 + t] = conj(Bt[t * 16 + p]);
            lower_solve(Lp, Nn + t, bp, 16);
            lower_h_solve(Lp, Nn + t, bp, 16);
        }
        __syncthreads();
        // Delta = alpha + sigma I - beta N
        for (int e = t; e < b * b; e += 64) {
            const int r = e / b, c = e - r * b;
            zd v = A[r * 16 + c];
            if (r == c) v.x += sg;
            for (int p = 0; p < bp; ++p) v = v - Bt[r * 16 + p] * Nn[p * 16 + c];
            Zs[r * 16 + c] = v;  // scratch
        }
        __syncthreads();
        for (int e = t; e < b * b; e += 64) {
            const int r = e / b, c = e - r * b;
            const zd v = Zs[r * 16 + c], w = conj(Zs[c * 16 + r]);
            D[r * 16 + c] = mk<double>(0.5 * (v.x + w.x), 0.5 * (v.y + w.y));
        }
    }
    __syncthreads();

    // Cholesky D = L L^H in place (lower triangle), right-looking.
    bool ok = true;
    for (int k = 0; k < b; ++k) {
        const double d = D[k * 16 + k].x;
        if (!(d > 0.0)) ok = false;
        const double rd = ok ? sqrt(d) : 1.0;
        __syncthreads();
        if (t == 0) D[k * 16 + k] = mk<double>(rd, 0.0);
        if (t > k && t < b) D[t * 16 + k] = zdivr(D[t * 16 + k], rd);
        __syncthreads();
        for (int e = t; e < b * b; e += 64) {
            const int r = e / b, c = e - r * b;
            if (c > k && r >= c) D[r * 16 + c] = D[r * 16 + c] - D[r * 16 + k] * conj(D[c * 16 + k]);
        }
        __syncthreads();
    }
    if (!ok) {
        if (t == 0) atomicOr(&rep->flags, kFlagNotHPD);
        return;
    }
    // keep the factor and N for the next step / the block update
    for (int e = t; e < b * b; e += 64) {
        const int r = e / b, c = e - r * b;
        st->L[j][r * 16 + c] = (c <= r) ? D[r * 16 + c] : mk<double>(0, 0);
    }
    if (!first) {
        for (int e = t; e < bp * b; e += 64) {
            const int r = e / b, c = e - r * b;
            st->N[j][r * 16 + c] = Nn[r * 16 + c];
        }
    }
    // M = Delta^{-1} Z: one column per lane
    for (int e = t; e < b * m; e += 64) {
        const int r = e / m, c = e - r * m;
        Zs[r * 16 + c] = st->Z[j][r * 16 + c];
    }
    __syncthreads();
    if (t < m) {
        lower_solve(D, Zs + t, b, 16);
        lower_h_solve(D, Zs + t, b, 16);
    }
    __syncthreads();
    for (int e = t; e < b * m; e += 64) {
        const int r = e / m, c = e - r * m;
        st->M[j][r * 16 + c] = Zs[r * 16 + c];
    }
}

hipError_t small_shift_coeffs(SmallState *st, StepReport *rep, const zd *alpha_raw, int first,
                              const int32_t *shift_list, int nact, hipStream_t stream) {
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(shift_coeffs_kernel, dim3(nact), dim3(64), 0, stream, st, rep, alpha_raw,
                       first, shift_list);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Window recurrences, applied after N_{j,i} and M_{j,i} of step i are known.  With Mh the columns of M_{j,i}
// still being updated:
//   first step of a window:  Wg = -N, Wfp = Wg Mh, Wh_0 = I, Wf_0 = Mh
//   later steps:             Wg <- -Wg N, Wfp += Wg Mh,
//                            Wh_u <- -Wh_u N, Wf_u += Wh_u Mh  (u < t),
//                            Wh_t = I, Wf_t = Mh
// (P_{j,i} = V_i - P_{j,i-1} N_{j,i} and X_j += P_{j,i} Mh unrolled over the window).
// ---------------------------------------------------------------------------
__device__ inline void mat_neg_mul(zd *A, const zd *N, int rows, int inner, int cols, zd *tmp) {
    // A (rows x inner) <- -A N (inner x cols), tmp: scratch of the same size in LDS
    const int t = threadIdx.x;
    for (int e = t; e < rows * cols; e += blockDim.x) {
        const int r = e / cols, c = e - r * cols;
        zd v = mk<double>(0, 0);
        for (int k = 0; k < inner; ++k) v = v - A[r * 16 + k] * N[k * 16 + c];
        tmp[r * 16 + c] = v;
    }
    __syncthreads();
    for (int e = t; e < 256; e += blockDim.x) {
        const int r = e / 16, c = e - r * 16;
        A[e] = (r < rows && c < cols) ? tmp[e] : mk<double>(0, 0);
    }
    __syncthreads();
}

__device__ inline void mat_mul_acc(zd *F, const zd *A, const zd *Mh, int rows, int inner, int cols,
                                   bool overwrite) {
    // F (rows x cols) (=|+=) A (rows x inner) Mh (inner x cols)
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
        const int r = e / 16, c = e - r * 16;
        zd v = mk<double>(0, 0);
        if (r < rows && c < cols)
            for (int k = 0; k < inner; ++k) v = v + A[r * 16 + k] * Mh[k * 16 + c];
        F[e] = overwrite ? v : F[e] + v;
    }
    __syncthreads();
}

size_t wincoef_bytes() {
    return sizeof(zd) * (2 * kS * 256 + 2 * (size_t)kS * kWinMax * 256) + sizeof(uint32_t) * kS +
           sizeof(int32_t) * kS;
}

WinCoef wincoef_at(void *base) {
    WinCoef w;
    zd *p = (zd *)base;
    w.Wg = p;
    w.Wfp = p + kS * 256;
    w.Wh = p + 2 * kS * 256;
    w.Wf = w.Wh + (size_t)kS * kWinMax * 256;
    w.Wmask = (uint32_t *)(w.Wf + (size_t)kS * kWinMax * 256);
    w.Wcount = (int32_t *)(w.Wmask + kS);
    return w;
}

// One block per (active shift, window slot); the slots are independent once
// N_{j,i} and M_{j,i} are known.  blockIdx.y = u < t: Wh_u <- -Wh_u N,
// Wf_u += Wh_u Mh; u == t: Wh_t = I, Wf_t = Mh; u == t + 1: the P_{j,i0}
// part (Wg, Wfp).
__global__ __launch_bounds__(64) void window_update_kernel(const SmallState *st, const StepReport *rep,
                                                           WinCoef wc, WindowStep w,
                                                           const int32_t *__restrict__ list) {
    __shared__ zd Ns[256], Mh[256], A[256], tmp[256];
    const int j = list[blockIdx.x];
    const int u = blockIdx.y;
    const int t = threadIdx.x;
    const uint32_t mask = rep->colmask[j];
    if (u == w.t + 1 && w.bp0 == 0) return;
    for (int e = t; e < 256; e += 64) {
        const int r = e / 16, c = e - r * 16;
        Ns[e] = st->N[j][e];
        Mh[e] = (r < w.b && c < w.m && ((mask >> c) & 1u)) ? st->M[j][e] : mk<double>(0, 0);
    }
    __syncthreads();
    if (u == w.t + 1) {
        zd *G = wc.Wg + j * 256, *Fp = wc.Wfp + j * 256;
        if (w.t == 0) {
            // Wg is the identity (b_{i0} x b_{i0}) at the window start, so Wg = -N
            for (int e = t; e < 256; e += 64) {
                const int r = e / 16, c = e - r * 16;
                A[e] = (r < w.bp0 && c < w.b) ? -Ns[e] : mk<double>(0, 0);
            }
            __syncthreads();
        } else {
            for (int e = t; e < 256; e += 64) A[e] = G[e];
            __syncthreads();
            mat_neg_mul(A, Ns, w.bp0, w.bp, w.b, tmp);
        }
        for (int e = t; e < 256; e += 64) {
            G[e] = A[e];
            tmp[e] = (w.t == 0) ? mk<double>(0, 0) : Fp[e];
        }
        __syncthreads();
        mat_mul_acc(tmp, A, Mh, w.bp0, w.b, w.m, false);
        for (int e = t; e < 256; e += 64) Fp[e] = tmp[e];
        return;
    }
    zd *H = wc.Wh + ((size_t)j * kWinMax + u) * 256, *F = wc.Wf + ((size_t)j * kWinMax + u) * 256;
    if (u == w.t) {
        for (int e = t; e < 256; e += 64) {
            const int r = e / 16, c = e - r * 16;
            H[e] = (r == c && r < w.b) ? mk<double>(1, 0) : mk<double>(0, 0);
            F[e] = Mh[e];
        }
        if (t == 0) {
            wc.Wmask[j] = (w.t == 0 ? 0u : wc.Wmask[j]) | mask;
            wc.Wcount[j] = w.t + 1;
        }
        return;
    }
    // rows of slot u beyond its width are zero, so all kS rows can be carried
    for (int e = t; e < 256; e += 64) A[e] = H[e];
    __syncthreads();
    mat_neg_mul(A, Ns, kS, w.bp, w.b, tmp);
    for (int e = t; e < 256; e += 64) {
        H[e] = A[e];
        tmp[e] = F[e];
    }
    __syncthreads();
    mat_mul_acc(tmp, A, Mh, kS, w.b, w.m, false);
    for (int e = t; e < 256; e += 64) F[e] = tmp[e];
}

hipError_t small_window_update(const SmallState *st, const StepReport *rep, WinCoef wc, WindowStep ws,
                               const int32_t *shift_list, int nact, hipStream_t stream) {
    if (nact <= 0) return hipSuccess;
    if (ws.t < 0 || ws.t >= kWinMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(window_update_kernel, dim3(nact, ws.t + 2), dim3(64), 0, stream, st, rep, wc, ws,
                       shift_list);
    return hipGetLastError();
}

__global__ void window_reset_kernel(WinCoef wc) {
    for (int j = threadIdx.x; j < kS; j += blockDim.x) {
        wc.Wmask[j] = 0u;
        wc.Wcount[j] = 0;
    }
}

hipError_t small_window_reset(WinCoef wc, hipStream_t stream) {
    hipLaunchKernelGGL(window_reset_kernel, dim3(1), dim3(64), 0, stream, wc);
    return hipGetLastError();
}

// One block of 64 lanes per (window shift, input pair, output tile): the
// lanes hold the matrix-core A operand, entry (output row i, input real
// index k) at lane i + 16 k.  With c the complex coefficient of input p
// in output q (out_q += in_p c):
//   Re out += Re in Re c - Im in Im c,   Im out += Re in Im c + Im in Re c.
template <typename R>
__global__ __launch_bounds__(64) void window_table_kernel(WinCoef wc, WindowTable wt,
                                                          const int32_t *__restrict__ shifts,
                                                          const int32_t *__restrict__ pmask, R *table) {
    const int js = blockIdx.x, pair = blockIdx.y, mt = blockIdx.z;
    const int lane = threadIdx.x;
    const int j = shifts[js];
    const int i = lane & 15, k = lane >> 4;
    // Output real column i of the tile: complex output q and its part po,
    // chosen so that each lane of the product ends with (re, im) of two
    // consecutive outputs in its four accumulators.  The f32 instruction
    // leaves rows 4 g + r of the result in lane group g, register r; the
    // f64 instruction leaves rows g + 4 r there.
    int ql, po;
    if (sizeof(R) == 8) {
        ql = 2 * (i & 3) + ((i >> 2) >> 1);
        po = (i >> 2) & 1;
    } else {
        ql = i >> 1;
        po = i & 1;
    }
    const int q = mt * 8 + ql;
    const int pin = k & 1;               // real/imaginary part of the input
    zd c = mk<double>(0, 0);
    const bool xout = q < wt.m;
    const bool pout = !xout && q - wt.m < wt.bend && pmask[j] != 0;
    if (xout || pout) {
        const int qq = xout ? q : q - wt.m;
        if (pair < wt.pairs_p) {
            const int p = 2 * pair + (k >> 1);
            if (p < wt.bp0) c = (xout ? wc.Wfp : wc.Wg)[j * 256 + p * 16 + qq];
        } else {
            const int col = 2 * (pair - wt.pairs_p) + (k >> 1);
            if (col < wt.ncolv) {
                // window slot u of this column and its first column c0
                int u = 0, c0 = 0;
                while (u < wt.K - 1 && col >= c0 + wt.wb[u]) c0 += wt.wb[u++];
                const int slot = wt.slot0 + u;
                if (slot < wc.Wcount[j]) {
                    const zd *src = (xout ? wc.Wf : wc.Wh) + ((size_t)j * kWinMax + slot) * 256;
                    c = src[(col - c0) * 16 + qq];
                }
            }
        }
    }
    const double v = (po == 0) ? (pin == 0 ? c.x : -c.y) : (pin == 0 ? c.y : c.x);
    table[(((size_t)js * wt.npairs + pair) * wt.nmt + mt) * 64 + lane] = (R)v;
}

hipError_t small_window_table(const WinCoef wc, const WindowTable &wt, const int32_t *shifts,
                              const int32_t *pmask, bool fp64, void *table, hipStream_t stream) {
    if (wt.nshift <= 0 || wt.npairs <= 0) return hipSuccess;
    if (wt.K < 1 || wt.slot0 < 0 || wt.slot0 + wt.K > kWinMax || wt.nmt < 1 || wt.nmt > 4)
        return hipErrorInvalidValue;
    const dim3 grid(wt.nshift, wt.npairs, wt.nmt);
    if (fp64)
        hipLaunchKernelGGL(window_table_kernel<double>, grid, dim3(64), 0, stream, wc, wt, shifts, pmask,
                           (double *)table);
    else
        hipLaunchKernelGGL(window_table_kernel<float>, grid, dim3(64), 0, stream, wc, wt, shifts, pmask,
                           (float *)table);
    return hipGetLastError();
}

// Three-product table (window3_kernel): one 64-lane block per (shift pair
// js2, block of 4 input columns).  Lane i + 16 k holds, for output row i of
// the matrix-core tile (two shifts of 8 outputs each) and input column
// 4 blk + k, the three real coefficients a, b and a + b of c = a + ib in
// table[((js2 * nblk + blk) * 3 + t) * 64 + lane], t = 0, 1, 2.  Row i
// belongs to register r of lane group g of the product (FP64 instruction:
// i = g + 4 r, FP32: i = 4 g + r), which stands for shift 2 js2 + (r >> 1)
// and output 2 g + (r & 1): both precisions leave the same output in the
// same register.
template <typename R>
__global__ __launch_bounds__(64) void window_table3_kernel(WinCoef wc, WindowTable wt,
                                                           const int32_t *__restrict__ shifts,
                                                           const int32_t *__restrict__ pmask, R *table) {
    const int js2 = blockIdx.x, blk = blockIdx.y;
    const int lane = threadIdx.x;
    const int i = lane & 15, k = lane >> 4;
    const int g = sizeof(R) == 8 ? (i & 3) : (i >> 2), r = sizeof(R) == 8 ? (i >> 2) : (i & 3);
    const int js = 2 * js2 + (r >> 1), q = 2 * g + (r & 1);
    const int col = 4 * blk + k;
    zd c = mk<double>(0, 0);
    if (js < wt.nshift && col < wt.ncolv) {
        const int j = shifts[js];
        const bool xout = q < wt.m;
        const bool pout = !xout && q - wt.m < wt.bend && pmask[j] != 0;
        if (xout || pout) {
            const int qq = xout ? q : q - wt.m;
            int u = 0, c0 = 0;
            while (u < wt.K - 1 && col >= c0 + wt.wb[u]) c0 += wt.wb[u++];
            const int slot = wt.slot0 + u;
            if (slot < wc.Wcount[j])
                c = (xout ? wc.Wf : wc.Wh)[((size_t)j * kWinMax + slot) * 256 + (col - c0) * 16 + qq];
        }
    }
    R *o = table + ((size_t)js2 * gridDim.y + blk) * 3 * 64 + lane;
    o[0] = (R)c.x;
    o[64] = (R)c.y;
    o[128] = (R)(c.x + c.y);
}

hipError_t small_window_table3(const WinCoef wc, const WindowTable &wt, const int32_t *shifts,
                               const int32_t *pmask, bool fp64, void *table, hipStream_t stream) {
    if (wt.nshift <= 0 || wt.ncolv <= 0) return hipSuccess;
    if (wt.K < 1 || wt.slot0 < 0 || wt.slot0 + wt.K > kWinMax || wt.bp0 != 0 || wt.m + wt.bend > 8 ||
        wt.nshift > 16)
        return hipErrorInvalidValue;
    const dim3 grid((wt.nshift + 1) / 2, (wt.ncolv + 3) / 4);
    if (fp64)
        hipLaunchKernelGGL(window_table3_kernel<double>, grid, dim3(64), 0, stream, wc, wt, shifts, pmask,
                           (double *)table);
    else
        hipLaunchKernelGGL(window_table3_kernel<float>, grid, dim3(64), 0, stream, wc, wt, shifts, pmask,
                           (float *)table);
    return hipGetLastError();
}

// One block of 64 lanes per (input pair, output tile) of the combined table.
template <typename R>
__global__ __launch_bounds__(64) void rational_table_kernel(WinCoef wc, WindowTable wt,
                                                            const int32_t *__restrict__ shifts,
                                                            const double *__restrict__ coef, R *table) {
    const int pair = blockIdx.x, mt = blockIdx.y;
    const int lane = threadIdx.x;
    const int i = lane & 15, k = lane >> 4;
    // output real i of the tile: complex output and part, ordered as in
    // window_table_kernel for the same instruction
    int ql, po;
    if (sizeof(R) == 8) {
        ql = 2 * (i & 3) + ((i >> 2) >> 1);
        po = (i >> 2) & 1;
    } else {
        ql = i >> 1;
        po = i & 1;
    }
    const int q = mt * 8 + ql;
    const int pin = k & 1;
    zd c = mk<double>(0, 0);
    if (q < wt.m) {
        const int npp = wt.nshift * wt.pairs_p;
        if (pair < npp) {
            const int js = pair / wt.pairs_p;
            const int p = 2 * (pair - js * wt.pairs_p) + (k >> 1);
            const int j = shifts[js];
            if (p < wt.bp0) {
                const zd f = wc.Wfp[j * 256 + p * 16 + q];
                c = mk<double>(coef[j] * f.x, coef[j] * f.y);
            }
        } else {
            const int col = 2 * (pair - npp) + (k >> 1);
            if (col < wt.ncolv) {
                int u = 0, c0 = 0;
                while (u < wt.K - 1 && col >= c0 + wt.wb[u]) c0 += wt.wb[u++];
                const int slot = wt.slot0 + u;
                for (int js = 0; js < wt.nshift; ++js) {
                    const int j = shifts[js];
                    if (slot < wc.Wcount[j]) {
                        const zd f = wc.Wf[((size_t)j * kWinMax + slot) * 256 + (col - c0) * 16 + q];
                        c.x += coef[j] * f.x;
                        c.y += coef[j] * f.y;
                    }
                }
            }
        }
    }
    const double v = (po == 0) ? (pin == 0 ? c.x : -c.y) : (pin == 0 ? c.y : c.x);
    table[((size_t)pair * gridDim.y + mt) * 64 + lane] = (R)v;
}

hipError_t small_rational_table(const WinCoef wc, const WindowTable &wt, const int32_t *shifts,
                                const double *coef, bool fp64, void *table, hipStream_t stream) {
    const int npairs = wt.nshift * wt.pairs_p + (wt.ncolv + 1) / 2;
    if (wt.nshift <= 0 || npairs <= 0) return hipSuccess;
    if (wt.K < 1 || wt.slot0 < 0 || wt.slot0 + wt.K > kWinMax || wt.m < 1 || wt.m > 16 ||
        wt.nshift > 16 || wt.pairs_p != (wt.bp0 + 1) / 2)
        return hipErrorInvalidValue;
    const dim3 grid(npairs, (wt.m + 7) / 8);
    if (fp64)
        hipLaunchKernelGGL(rational_table_kernel<double>, grid, dim3(64), 0, stream, wc, wt, shifts, coef,
                           (double *)table);
    else
        hipLaunchKernelGGL(rational_table_kernel<float>, grid, dim3(64), 0, stream, wc, wt, shifts, coef,
                           (float *)table);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// alpha_i = herm(raw Gram); coef[1] = -alpha_i for the block combination.
// ---------------------------------------------------------------------------
__global__ void prep_alpha_kernel(SmallState *st, const zd *__restrict__ raw) {
    const int b = st->b;
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
        const int r = e / 16, c = e - r * 16;
        zd h = mk<double>(0, 0);
        if (r < b && c < b) {
            const zd v = raw[r * 16 + c], w = conj(raw[c * 16 + r]);
            h = mk<double>(0.5 * (v.x + w.x), 0.5 * (v.y + w.y));
        }
        st->alpha[e] = h;
        st->coef[1][e] = -h;
    }
}

hipError_t small_prep_alpha(SmallState *st, const zd *alpha_raw, hipStream_t stream) {
    hipLaunchKernelGGL(prep_alpha_kernel, dim3(1), dim3(256), 0, stream, st, alpha_raw);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// First CholQR pass with deflation (single thread: b <= 16).
// Column k of W is kept when the Schur remainder d_k of W^H W exceeds
// (tau_W ||T||_est)^2; R1 gets one row per kept column.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void chol_deflate_kernel(SmallState *st, StepReport *rep,
                                                          const zd *__restrict__ alpha_raw,
                                                          const zd *__restrict__ G, double tau_W,
                                                          const zd *__restrict__ Gref) {
    // The inputs go to LDS with every lane.  The factorisation runs column by
    // column: thread 0 forms the remainder d of column k and decides, and
    // when k is kept the other lanes form its row of R for the columns after
    // k at once (each entry by the same formula, in the same order, as a
    // column-by-column solve); the inverse columns and the conditioning terms
    // then run one per lane.
    __shared__ zd Gs[256], R[256], C1s[256];
    __shared__ double nrm[2], gref[16], dterm[16], thr_s;
    __shared__ int piv[16], nks, skip, keepk, unresolved;
    const int t = threadIdx.x;
    const int b = st->b, bp = st->bp;
    (void)alpha_raw;
    if (t < 16) gref[t] = (Gref ? Gref : G)[t * 16 + t].x;
    // ||T||_est from alpha_i and beta_i
    double na = 0.0, nb = 0.0;
    for (int e = t; e < 256; e += 64) {
        Gs[e] = G[e];
        const int r = e / 16, c = e - r * 16;
        if (r < b && c < b) na += norm2(st->alpha[e]);
        if (r < b && c < bp) nb += norm2(st->beta[e]);
        R[e] = mk<double>(0, 0);
        C1s[e] = mk<double>(0, 0);
    }
    for (int off = 32; off > 0; off >>= 1) {
        na += __shfl_xor(na, off, 64);
        nb += __shfl_xor(nb, off, 64);
    }
    if (t == 0) {
        nrm[0] = na;
        nrm[1] = nb;
    }
    __syncthreads();
    if (t == 0) {
        double test = st->test;
        test = fmax(test, sqrt(nrm[0]));
        test = fmax(test, sqrt(nrm[1]));
        st->test = test;
        thr_s = tau_W * test;
        nks = 0;
        unresolved = 0;
    }
    __syncthreads();
    const double thr = thr_s;
    for (int k = 0; k < b; ++k) {
        if (t == 0) {
            const int nk = nks;
            const double gkk = fmax(Gs[k * 16 + k].x, gref[k]);  // scale of the rounding of d
            double d = Gs[k * 16 + k].x;
            for (int r = 0; r < nk; ++r) d -= norm2(R[r * 16 + k]);
            // a remainder at the rounding level of G_kk decides nothing when
            // the threshold lies below that level
            if (d <= kResolve * gkk && kResolve * gkk > thr * thr) unresolved = 1;
            keepk = 0;
            if (d > thr * thr) {
                // a kept column: new row nk of R (dropped columns keep the
                // entries of the rows above)
                R[nk * 16 + k] = mk<double>(sqrt(d), 0.0);
                piv[nk] = k;
                nks = nk + 1;
                keepk = 1;
            }
        }
        __syncthreads();
        if (keepk) {
            const int r = nks - 1, c = k + 1 + t;
            if (c < b) {
                zd v = Gs[k * 16 + c];
                for (int q = 0; q < r; ++q) v = v - conj(R[q * 16 + k]) * R[q * 16 + c];
                R[r * 16 + c] = zdivr(v, R[r * 16 + k].x);
            }
        }
        __syncthreads();
    }
    const int nk = nks;
    // C1 = E_K R_KK^{-1}: R_KK (nk x nk) is R restricted to the pivot
    // columns; column q of R_KK^{-1} solves R_KK x = e_q (upper triangular)
    if (t < nk) {
        const int q = t;
        zd x[16];
        for (int r = nk - 1; r >= 0; --r) {
            zd v = (r == q) ? mk<double>(1, 0) : mk<double>(0, 0);
            for (int c = r + 1; c < nk; ++c) v = v - R[r * 16 + piv[c]] * x[c];
            x[r] = zdivr(v, R[r * 16 + piv[r]].x);
        }
        for (int r = 0; r < nk; ++r) C1s[piv[r] * 16 + q] = x[r];
    }
    __syncthreads();
    // condition of the kept columns scaled to unit norm, Rs = R_KK D^{-1}:
    // ||Rs||_F^2 = nk and Rs^{-1} = D R_KK^{-1} (rows scaled by the norms)
    if (t < nk) {
        const int c = t;
        double d2 = 0.0;
        for (int r = 0; r <= c; ++r) d2 += norm2(R[r * 16 + piv[c]]);
        double row2 = 0.0;
        for (int q = 0; q < nk; ++q) row2 += norm2(C1s[piv[c] * 16 + q]);
        dterm[c] = d2 * row2;
    }
    __syncthreads();
    if (t == 0) {
        double inv2 = 0.0;
        for (int c = 0; c < nk; ++c) inv2 += dterm[c];
        skip = (nk > 0 && nk * inv2 <= 16.0 * 16.0) ? 1 : 0;
        st->redo = unresolved;
        if (unresolved) {
            skip = 1;
            rep->flags |= kFlagRedoQR;
        }
    }
    __syncthreads();
    for (int e = t; e < 256; e += 64) {
        const int r = e / 16;
        if (r < nk) st->R1[e] = R[e];
        st->C1[e] = C1s[e];
    }
    if (t < 16) rep->kept[t] = (t < nk) ? piv[t] : -1;
    if (t == 0) {
        st->skip_qr2 = skip;
        rep->skip_qr2 = skip;
        rep->bnew = nk;
    }
}

hipError_t small_chol_deflate(SmallState *st, StepReport *rep, const zd *alpha_raw, const zd *G,
                              double tau_W, hipStream_t stream, const zd *Gref) {
    hipLaunchKernelGGL(chol_deflate_kernel, dim3(1), dim3(64), 0, stream, st, rep, alpha_raw, G,
                       tau_W, Gref);
    return hipGetLastError();
}

// G = G' - M^H alpha - alpha^H M + alpha^H alpha, hermitised (b x b).
__global__ __launch_bounds__(256) void lanczos_gram_kernel(const SmallState *st, const zd *__restrict__ M,
                                                           const zd *__restrict__ Gp, zd *__restrict__ G) {
    __shared__ zd Ms[256], As[256], NA[256], T[256];
    const int t = threadIdx.x;
    const int b = st->b;
    Ms[t] = M[t];
    As[t] = st->alpha[t];
    __syncthreads();
    const int r = t / 16, c = t - r * 16;
    // N alpha
    zd na = mk<double>(0, 0);
    if (r < b && c < b)
        for (int k = 0; k < b; ++k) na = na + st->Nv[r * 16 + k] * As[k * 16 + c];
    NA[t] = na;
    __syncthreads();
    zd v = mk<double>(0, 0);
    if (r < b && c < b) {
        v = Gp[t];
        for (int k = 0; k < b; ++k) {
            // (M^H alpha)_{rc} = sum_k conj(M_kr) alpha_kc, (alpha^H M)_{rc} = sum_k conj(alpha_kr) M_kc
            v = v - conj(Ms[k * 16 + r]) * As[k * 16 + c] - conj(As[k * 16 + r]) * Ms[k * 16 + c] +
                conj(As[k * 16 + r]) * NA[k * 16 + c];
        }
    }
    T[t] = v;
    __syncthreads();
    const zd w = conj(T[c * 16 + r]);
    G[t] = mk<double>(0.5 * (v.x + w.x), 0.5 * (v.y + w.y));
}

hipError_t small_lanczos_gram(const SmallState *st, const zd *M, const zd *Gp, zd *G, hipStream_t stream) {
    hipLaunchKernelGGL(lanczos_gram_kernel, dim3(1), dim3(256), 0, stream, st, M, Gp, G);
    return hipGetLastError();
}

__global__ void set_nv_kernel(SmallState *st, const zd *__restrict__ G) {
    const int b = st->b;
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
        const int r = e / 16, c = e - r * 16;
        st->Nv[e] = (r < b && c < b) ? G[e] : mk<double>(0, 0);
    }
}

hipError_t small_set_nv(SmallState *st, const zd *G, hipStream_t stream) {
    hipLaunchKernelGGL(set_nv_kernel, dim3(1), dim3(256), 0, stream, st, G);
    return hipGetLastError();
}

// cB[0] = C1, cB[1] = coef[1] C1 (-alpha C1), cB[2] = coef[0] C1 (-beta^H C1).
__global__ __launch_bounds__(256) void basis_coefs_kernel(SmallState *st) {
    __shared__ zd C1s[256];
    const int t = threadIdx.x;
    if (st->redo) return;  // uniform: the basis is formed column by column instead
    const int b = st->b;
    C1s[t] = st->C1[t];
    __syncthreads();
    const int r = t / 16, c = t - r * 16;
    zd va = mk<double>(0, 0), vb = mk<double>(0, 0);
    for (int k = 0; k < b; ++k) {
        va = va + st->coef[1][r * 16 + k] * C1s[k * 16 + c];
        vb = vb + st->coef[0][r * 16 + k] * C1s[k * 16 + c];
    }
    st->cB[0][t] = C1s[t];
    st->cB[1][t] = va;
    st->cB[2][t] = vb;
}

hipError_t small_basis_coefs(SmallState *st, hipStream_t stream) {
    hipLaunchKernelGGL(basis_coefs_kernel, dim3(1), dim3(256), 0, stream, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Second CholQR pass, beta_{i+1}, residual coefficients and freezing.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void finish_kernel(SmallState *st, StepReport *rep,
                                                     const zd *__restrict__ G2, double tol,
                                                     int freeze, const int32_t *__restrict__ list,
                                                     int nact) {
    __shared__ zd R2[256], BN[256], G2s[256], R1s[256];
    __shared__ int fail;
    if (st->redo) return;  // uniform: the QR of this step is redone first
    const int t = threadIdx.x;
    const int b = st->b, m = st->m;
    const int nk = rep->bnew;
    const int skip = st->skip_qr2;
    // inputs to LDS with every lane; the sequential part below reads LDS only
    for (int e = t; e < 256; e += blockDim.x) {
        G2s[e] = skip ? mk<double>(0, 0) : G2[e];
        R1s[e] = st->R1[e];
        R2[e] = mk<double>(0, 0);
    }
    __syncthreads();
    if (t == 0) {
        fail = 0;
        // G2 = R2^H R2, R2 upper triangular (nk x nk); R2 = I when the
        // second pass was not run
        if (skip)
            for (int k = 0; k < nk; ++k) R2[k * 16 + k] = mk<double>(1, 0);
        for (int k = 0; k < nk && !skip; ++k) {
            double d = G2s[k * 16 + k].x;
            for (int q = 0; q < k; ++q) d -= norm2(R2[q * 16 + k]);
            if (!(d > 0.0)) {
                fail = 1;
                d = 1.0;
            }
            const double rd = sqrt(d);
            R2[k * 16 + k] = mk<double>(rd, 0.0);
            for (int c = k + 1; c < nk; ++c) {
                zd v = G2s[k * 16 + c];
                for (int q = 0; q < k; ++q) v = v - conj(R2[q * 16 + k]) * R2[q * 16 + c];
                R2[k * 16 + c] = zdivr(v, rd);
            }
        }
        if (fail) atomicOr(&rep->flags, kFlagQR2);
    }
    __syncthreads();
    // R2inv = R2^{-1}: row r of I solved against upper-triangular R2, one
    // row per thread
    if (t < 16) {
        const int r = t;
        zd x[16];
        for (int c = 0; c < nk; ++c) {
            zd v = (r == c) ? mk<double>(1, 0) : mk<double>(0, 0);
            for (int q = 0; q < c; ++q) v = v - x[q] * R2[q * 16 + c];
            x[c] = zdivr(v, R2[c * 16 + c].x);
        }
        for (int c = 0; c < 16; ++c) st->R2inv[r * 16 + c] = (r < nk && c < nk) ? x[c] : mk<double>(0, 0);
    }
    // beta_{i+1} = R2 R1 (nk x b), one entry per thread
    {
        const int r = t >> 4, c = t & 15;
        zd v = mk<double>(0, 0);
        if (r < nk && c < b)
            for (int q = r; q < nk; ++q) v = v + R2[r * 16 + q] * R1s[q * 16 + c];
        BN[r * 16 + c] = v;
    }
    __syncthreads();
    // per shift and column l: column l of C_j = -beta_{i+1} M_j = Z_{j,i+1};
    // its estimate; freezing (each thread clears only its own bit)
    for (int w = t; w < nact * m; w += 256) {
        const int js = w / m, l = w - js * m;
        const int j = list[js];
        double nrm = 0.0;
        for (int r = 0; r < nk; ++r) {
            zd v = mk<double>(0, 0);
            for (int q = 0; q < b; ++q) v = v - BN[r * 16 + q] * st->M[j][q * 16 + l];
            st->Z[j][r * 16 + l] = v;
            nrm += norm2(v);
        }
        const double bn = st->bnorm[st->colmap[j][l]];
        const double e = (bn > 0.0) ? sqrt(nrm) / bn : 0.0;
        rep->est[j][l] = e;
        if (freeze && ((rep->colmask[j] >> l) & 1u) && e <= tol) atomicAnd(&rep->colmask[j], ~(1u << l));
    }
    __syncthreads();
    for (int e = t; e < 256; e += 256) {
        const int r = e / 16, c = e - r * 16;
        // Gram of V_{i+1} as stored: the measured one when it was not
        // re-orthonormalised (entries past the new width are zero)
        st->Nv[e] = skip ? ((r < nk && c < nk) ? G2[e] : mk<double>(0, 0))
                         : ((r == c && r < nk) ? mk<double>(1, 0) : mk<double>(0, 0));
        st->betanext[e] = BN[e];
        st->beta[e] = BN[e];
        // -beta_{i+1}^H (b x bnew): coefficient of V_i in the next step
        st->coef[0][e] = -conj(BN[c * 16 + r]);
    }
    if (t == 0) {
        st->bp = b;
        st->b = nk;
    }
}

hipError_t small_finish(SmallState *st, StepReport *rep, const zd *G2, double tol, int freeze,
                        const int32_t *shift_list, int nact, hipStream_t stream) {
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, stream, st, rep, G2, tol, freeze,
                       shift_list, nact);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Vector-wise stopping (Sec. 3: the iterates advance one Lanczos vector at a
// time).  The leading part of a block root-free Cholesky factorisation of
// T_sigma is the factorisation of its leading part, so within block step i
// (width b, K_{i-1} vectors before it) the Galerkin iterate on the first
// K_{i-1} + r vectors is
//   X^(r) = X_{i-1} + P_{j,i}[:, 1..r] y_r,   y_r = Delta_r^{-1} Z_{j,i}[1..r]
// (Delta_r the leading r x r part of Delta_{j,i}), and its residual is
// V_i[:, r+1..b] c_a + V_{i+1} c_b with
//   c_a = Z_{j,i}[r+1..b] - Delta_{j,i}[r+1..b, 1..r] y_r,   c_b = -beta_{i+1}[:, 1..r] y_r
// (Z_{j,1} = rho covers the first block).  With Delta_{j,i} = L L^H and
// w = L^{-1} Z_{j,i} = L^H M_{j,i} these are
//   y_r = L_r^{-H} w[1..r],   c_a[a] = sum_{k = r+1..a} L[a][k] w[k].
// r = b is the block iterate, whose estimate small_finish has computed.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void vector_stop_kernel(SmallState *st, StepReport *rep, double tol,
                                                          const int32_t *__restrict__ list, int nact) {
    __shared__ uint32_t mask[kS];
    if (st->redo) return;  // uniform: the QR of this step is redone first
    const int t = threadIdx.x;
    const int b = st->bp, nk = st->b, m = st->m;  // small_finish has rotated the widths
    const int js = t / kS, l = t - js * kS;
    const bool mine = js < nact && l < m;
    const int j = mine ? list[js] : 0;
    if (t < nact) mask[t] = rep->colmask[list[t]];
    __syncthreads();
    int rstop = 0;
    double estop = 0.0;
    zd y[kS];
    if (mine) {
        for (int q = 0; q < kS; ++q) st->dM[j][q * 16 + l] = mk<double>(0, 0);
        rep->stage[j][l] = 0;
    }
    if (mine && ((mask[js] >> l) & 1u)) {
        const zd *L = st->L[j];
        const zd *M = st->M[j];
        const zd *BN = st->betanext;
        const double bn = st->bnorm[st->colmap[j][l]];
        zd w[kS];
        for (int a = 0; a < b; ++a) {
            zd v = mk<double>(0, 0);
            for (int k = a; k < b; ++k) v = v + conj(L[k * 16 + a]) * M[k * 16 + l];
            w[a] = v;
        }
        for (int r = 1; r < b && !rstop; ++r) {
            double na = 0.0;
            for (int a = r; a < b; ++a) {
                zd v = mk<double>(0, 0);
                for (int k = r; k <= a; ++k) v = v + L[a * 16 + k] * w[k];
                na += norm2(v);
            }
            for (int q = r - 1; q >= 0; --q) {
                zd v = w[q];
                for (int c = q + 1; c < r; ++c) v = v - conj(L[c * 16 + q]) * y[c];
                y[q] = zdivr(v, L[q * 16 + q].x);
            }
            double nb = 0.0;
            for (int q = 0; q < nk; ++q) {
                zd v = mk<double>(0, 0);
                for (int k = 0; k < r; ++k) v = v + BN[q * 16 + k] * y[k];
                nb += norm2(v);
            }
            const double e = (bn > 0.0) ? sqrt(na + nb) / bn : 0.0;
            if (e <= tol) {
                rstop = r;
                estop = e;
            }
        }
        if (!rstop && rep->est[j][l] <= tol) {
            rstop = b;
            estop = rep->est[j][l];
        }
        if (rstop) {
            atomicAnd(&mask[js], ~(1u << l));
            rep->est[j][l] = estop;
            rep->stage[j][l] = rstop;
            if (rstop < b)
                for (int q = 0; q < b; ++q)
                    st->dM[j][q * 16 + l] = (q < rstop ? y[q] : mk<double>(0, 0)) - M[q * 16 + l];
        }
    }
    __syncthreads();
    if (t < nact) rep->colmask[list[t]] = mask[t];
}

hipError_t small_vector_stop(SmallState *st, StepReport *rep, double tol, const int32_t *shift_list,
                             int nact, hipStream_t stream) {
    if (nact <= 0) return hipSuccess;
    if (nact > kS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(vector_stop_kernel, dim3(1), dim3(256), 0, stream, st, rep, tol, shift_list, nact);
    return hipGetLastError();
}

// One block per (active shift, window slot), as window_update_kernel.
__global__ __launch_bounds__(64) void window_correct_kernel(const SmallState *st, WinCoef wc, WindowStep w,
                                                            const int32_t *__restrict__ list) {
    __shared__ zd Mh[256], A[256], tmp[256];
    if (st->redo) return;
    const int j = list[blockIdx.x];
    const int u = blockIdx.y;
    const int t = threadIdx.x;
    if (u == w.t + 1 && w.bp0 == 0) return;
    for (int e = t; e < 256; e += 64) {
        const int r = e / 16, c = e - r * 16;
        Mh[e] = (r < w.b && c < w.m) ? st->dM[j][e] : mk<double>(0, 0);
    }
    __syncthreads();
    if (u == w.t + 1) {
        zd *G = wc.Wg + j * 256, *Fp = wc.Wfp + j * 256;
        for (int e = t; e < 256; e += 64) {
            A[e] = G[e];
            tmp[e] = Fp[e];
        }
        __syncthreads();
        mat_mul_acc(tmp, A, Mh, w.bp0, w.b, w.m, false);
        for (int e = t; e < 256; e += 64) Fp[e] = tmp[e];
        return;
    }
    zd *H = wc.Wh + ((size_t)j * kWinMax + u) * 256, *F = wc.Wf + ((size_t)j * kWinMax + u) * 256;
    if (u == w.t) {
        for (int e = t; e < 256; e += 64) F[e] = F[e] + Mh[e];
        return;
    }
    for (int e = t; e < 256; e += 64) {
        A[e] = H[e];
        tmp[e] = F[e];
    }
    __syncthreads();
    mat_mul_acc(tmp, A, Mh, kS, w.b, w.m, false);
    for (int e = t; e < 256; e += 64) F[e] = tmp[e];
}

hipError_t small_window_correct(const SmallState *st, WinCoef wc, WindowStep ws, const int32_t *shift_list,
                                int nact, hipStream_t stream) {
    if (nact <= 0) return hipSuccess;
    if (ws.t < 0 || ws.t >= kWinMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(window_correct_kernel, dim3(nact, ws.t + 2), dim3(64), 0, stream, st, wc, ws,
                       shift_list);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Column-by-column deflated QR of W, used when the first CholQR pass cannot
// resolve a drop decision (classical Gram-Schmidt twice, column order).
// ---------------------------------------------------------------------------
__global__ void wqr_begin_kernel(SmallState *st) {
    for (int e = threadIdx.x; e < 256; e += blockDim.x) st->R1[e] = mk<double>(0, 0);
}

hipError_t small_wqr_begin(SmallState *st, hipStream_t stream) {
    hipLaunchKernelGGL(wqr_begin_kernel, dim3(1), dim3(256), 0, stream, st);
    return hipGetLastError();
}

__global__ void wqr_decide_kernel(SmallState *st, StepReport *rep, const zd *__restrict__ c1,
                                  const zd *__restrict__ c2, const zd *__restrict__ nu2, int k, int l,
                                  double tau) {
    if (threadIdx.x != 0) return;
    for (int r = 0; r < k; ++r) {
        const zd a = c1 ? c1[r * 16] : mk<double>(0, 0);
        const zd bb = c2 ? c2[r * 16] : mk<double>(0, 0);
        st->R1[r * 16 + l] = a + bb;
    }
    const double nu = sqrt(fmax(nu2[0].x, 0.0));
    const bool keep = nu > tau * st->test;
    if (keep) st->R1[k * 16 + l] = mk<double>(nu, 0.0);
    st->coef[3][0] = mk<double>(keep ? 1.0 / nu : 0.0, 0.0);
    rep->scalar[0] = nu;
    rep->scalar[1] = keep ? 1.0 : 0.0;
}

hipError_t small_wqr_decide(SmallState *st, StepReport *rep, const zd *c1, const zd *c2, const zd *nu2,
                            int k, int l, double tau, hipStream_t stream) {
    if (k < 0 || k >= kS || l < 0 || l >= kS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wqr_decide_kernel, dim3(1), dim3(64), 0, stream, st, rep, c1, c2, nu2, k, l, tau);
    return hipGetLastError();
}

__global__ void wqr_end_kernel(SmallState *st, StepReport *rep, int nk, WqrKept kept) {
    const int t = threadIdx.x;
    if (t < kS) rep->kept[t] = (t < nk) ? kept.col[t] : -1;
    if (t == 0) {
        // beta_{i+1} = R1: the second pass is not run, and finish_kernel
        // takes R2 = I
        st->skip_qr2 = 1;
        rep->skip_qr2 = 1;
        rep->bnew = nk;
        st->redo = 0;
        rep->flags &= ~kFlagRedoQR;
    }
}

hipError_t small_wqr_end(SmallState *st, StepReport *rep, int nk, WqrKept kept, hipStream_t stream) {
    if (nk < 0 || nk > kS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wqr_end_kernel, dim3(1), dim3(64), 0, stream, st, rep, nk, kept);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Initial deflated QR of B (classical Gram-Schmidt twice, column order).
// ---------------------------------------------------------------------------
__global__ void bnorms_kernel(SmallState *st, StepReport *rep, const zd *__restrict__ G, int c0,
                              int cnt) {
    if (threadIdx.x != 0) return;
    for (int l = 0; l < cnt; ++l) {
        const double v = G[l * 16 + l].x;
        if (!isfinite(v)) rep->flags |= kFlagNonFinite;
        st->bnorm[c0 + l] = sqrt(fmax(v, 0.0));
        for (int r = 0; r < kS; ++r) st->rho[r * kStack + c0 + l] = mk<double>(0, 0);
    }
}

hipError_t small_bnorms(SmallState *st, StepReport *rep, const zd *G, int c0, int cnt,
                        hipStream_t stream) {
    hipLaunchKernelGGL(bnorms_kernel, dim3(1), dim3(64), 0, stream, st, rep, G, c0, cnt);
    return hipGetLastError();
}

__global__ void neg_column_kernel(SmallState *st, int slot, const zd *__restrict__ src, int k) {
    const int t = threadIdx.x;
    if (t < 16) st->coef[slot][t * 16] = (t < k) ? -src[t * 16] : mk<double>(0, 0);
}

hipError_t small_neg_column(SmallState *st, int slot, const zd *src, int k, hipStream_t stream) {
    hipLaunchKernelGGL(neg_column_kernel, dim3(1), dim3(64), 0, stream, st, slot, src, k);
    return hipGetLastError();
}

__global__ void cgs_decide_kernel(SmallState *st, StepReport *rep, const zd *__restrict__ c1,
                                  const zd *__restrict__ c2, const zd *__restrict__ nu2, int k,
                                  int l, double tau_B) {
    if (threadIdx.x != 0) return;
    for (int r = 0; r < k; ++r) {
        const zd a = c1 ? c1[r * 16] : mk<double>(0, 0);
        const zd bb = c2 ? c2[r * 16] : mk<double>(0, 0);
        st->rho[r * kStack + l] = a + bb;
    }
    const double nu = sqrt(fmax(nu2[0].x, 0.0));
    bool keep = nu > tau_B * st->bnorm[l];
    if (keep && k >= kS) {
        rep->flags |= kFlagRank;
        keep = false;
    }
    if (keep) st->rho[k * kStack + l] = mk<double>(nu, 0.0);
    st->coef[3][0] = mk<double>(keep ? 1.0 / nu : 0.0, 0.0);
    rep->scalar[0] = nu;
    rep->scalar[1] = keep ? 1.0 : 0.0;
}

hipError_t small_cgs_decide(SmallState *st, StepReport *rep, const zd *c1, const zd *c2,
                            const zd *nu2, int k, int l, double tau_B, hipStream_t stream) {
    hipLaunchKernelGGL(cgs_decide_kernel, dim3(1), dim3(64), 0, stream, st, rep, c1, c2, nu2, k, l,
                       tau_B);
    return hipGetLastError();
}

struct ShiftInit {
    double sigma[kS];
};

__global__ void init_shifts_kernel(SmallState *st, StepReport *rep, int m1, int m, int s,
                                   ShiftInit sh, int freeze, double tol, int per_shift) {
    if (threadIdx.x != 0) return;
    st->b = m1;
    st->bp = 0;
    st->m = m;
    st->s = s;
    st->test = 0.0;
    st->redo = 0;
    st->skip_qr2 = 0;
    for (int e = 0; e < 256; ++e) st->Nv[e] = mk<double>((e / 16 == e % 16) ? 1.0 : 0.0, 0.0);
    for (int e = 0; e < 256; ++e) st->beta[e] = mk<double>(0, 0);
    for (int j = 0; j < s; ++j) {
        st->sigma[j] = sh.sigma[j];
        for (int e = 0; e < 256; ++e) st->Z[j][e] = mk<double>(0, 0);
        uint32_t mask = 0;
        for (int l = 0; l < m; ++l) {
            const int c = per_shift ? j * m + l : l;
            st->colmap[j][l] = c;
            double nrm = 0.0;
            for (int r = 0; r < m1; ++r) {
                const zd v = st->rho[r * kStack + c];
                st->Z[j][r * 16 + l] = v;
                nrm += norm2(v);
            }
            const double bn = st->bnorm[c];
            const double e = bn > 0.0 ? sqrt(nrm) / bn : 0.0;
            rep->est[j][l] = e;
            if (bn > 0.0 && !(freeze && e <= tol)) mask |= 1u << l;
        }
        rep->colmask[j] = mask;
    }
    rep->bnew = m1;
}

hipError_t small_init_shifts(SmallState *st, StepReport *rep, int m1, int m, int s,
                             const double *sigma_host, int freeze, double tol, int per_shift,
                             hipStream_t stream) {
    ShiftInit sh{};
    for (int j = 0; j < s && j < kS; ++j) sh.sigma[j] = sigma_host[j];
    hipLaunchKernelGGL(init_shifts_kernel, dim3(1), dim3(64), 0, stream, st, rep, m1, m, s, sh,
                       freeze, tol, per_shift);
    return hipGetLastError();
}

}  // namespace dsbcg
