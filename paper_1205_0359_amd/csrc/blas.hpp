// Tall-skinny block kernels: combinations X C, Gram products X^H Y, the
// per-shift P / X updates and layout conversions.
#pragma once

#include "common.hpp"

namespace dsbcg {

constexpr int kMaxW = 16;       // largest block width (right-hand sides, shifts)
constexpr int kTsThreads = 256; // threads of a tall-skinny workgroup

// A tall-skinny matrix is nrows x b, row-major with leading dimension ld.
struct TsArgs {
    int64_t nrows;
    int K;                      // inputs combined: out = sum_k X_k C_k
    const void *X[3];
    int64_t ldx[3];
    int bx[3];
    const zd *C[3];             // FP64 [bx][bout] row-major, leading dimension 16; NULL = identity
    int bout;
    void *out;                  // optional store of the combination
    int64_t ldo;
    int gram;                   // 0: none, 1: partial out^H out, 2: partial L^H out
    const void *L;
    int64_t ldl;
    int bl;
    zd *partials;               // [nwg][16*16] FP64 partial Gram matrices
    int64_t rows_per_wg;
};

// Launch the combination / Gram kernel on `nwg` workgroups.
hipError_t ts_run(bool fp64, TsArgs a, int nwg, hipStream_t st);

// out[e] = sum_w partials[w][e] for e < nelem, summed in a fixed order.
hipError_t reduce_partials(const zd *partials, int nwg, int nelem, zd *out, hipStream_t st);

// Row orderings of an n x b field (n = 12 V):
//   kPlane: row = c * V + x   (spin-colour plane, then site)
//   kApi:   row = x * 12 + c  (site, then spin-colour)  == [V][4][3][b]
enum RowOrder { kPlane = 0, kApi = 1 };

// out (To) [row'][col] (=|+=) scale * in (Ti) [row][col_in0 + col] for cols columns.
hipError_t copy_field(bool in_fp64, bool out_fp64, int64_t V, int cols, const void *in,
                      int64_t in_ld, int in_order, int in_col0, void *out, int64_t out_ld,
                      int out_order, bool accumulate, double scale, hipStream_t st);

// Per-shift update of Sec. 3 in block form, for the listed shifts j:
//   P_j <- V_i - P_j N_j      (or P_j <- V_i on the first step)
//   X_j[:, l] += P_j M_j[:, l] for the columns l set in colmask[j]
// V: n x b (ld b); P old: ld bp, P new: ld b (separate buffers); X: ld m.
struct ShiftArgs {
    int64_t nrows;
    const void *V;
    int b, bp, m;
    const void *Pold;           // [s][n][bp]
    void *Pnew;                 // [s][n][b]
    int64_t pstride;            // elements between shifts in P buffers
    void *X;                    // [s][n][m]
    int64_t xstride;
    const void *N;              // [s][16*16] coefficients in the data precision
    const void *M;              // [s][16*16]
    const int32_t *shifts;      // device list of shift indices
    int nshift;
    const uint32_t *colmask;    // device [s] active-column bit masks
    int first;
};
hipError_t shift_update(bool fp64, const ShiftArgs &a, hipStream_t st);

// Checks a field for NaN/Inf: sets *flag (device int) to 1 if any is found.
hipError_t find_nonfinite(const double *data, int64_t count, int32_t *flag, hipStream_t st);

}  // namespace dsbcg
