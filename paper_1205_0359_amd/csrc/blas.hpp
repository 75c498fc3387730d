// Tall-skinny block kernels: combinations X C, Gram products X^H Y, the
// per-shift P / X updates and layout conversions.
//
// A block of b columns is column-major: element (row, column q) at
// q * cs + row, cs >= nrows the column stride.  For a lattice field the row
// index is c * V + x (spin-colour c, site x).
#pragma once

#include "common.hpp"

namespace dsbcg {

constexpr int kMaxW = 16;  // largest block width (right-hand sides, shifts)

struct TsArgs {
    int64_t nrows;
    int K;                   // inputs combined: out = sum_k X_k C_k
    const void *X[3];
    int64_t cs[3];           // column strides
    int bx[3];
    const zd *C[3];          // FP64 [bx][bout] row-major, leading dimension 16; NULL = identity
    int bout;
    void *out;               // optional store of the combination
    int64_t cso;
    int gram;                // 0: none, 1: partial out^H out, 2: partial L^H out
    const void *L;
    int64_t csl;
    int bl;
    zd *partials;            // [nwg][16*16] FP64 partial Gram matrices
    int64_t rows_per_wg;
};

// Launch the combination / Gram kernel; *nwg receives the workgroup count
// whose partials must be reduced (at most max_wg).
hipError_t ts_run(bool fp64, TsArgs a, int max_wg, int *nwg, hipStream_t st);

// out[e] = sum_w partials[w][e] for e < nelem, summed in a fixed order.
hipError_t reduce_partials(const zd *partials, int nwg, int nelem, zd *out, hipStream_t st);

// A lattice field of `cols` columns in one of two layouts:
//   kApi: [V][12][ld] with the columns at col0 .. col0+cols-1 of each row
//   kCM:  column-major, element (x, c, r) at r * cs + c * V + x
enum FieldLayout { kCM = 0, kApi = 1 };
struct FieldDesc {
    void *p;
    int layout;
    int64_t ld;   // kApi: row length; kCM: column stride
    int col0;     // kApi: first column
    bool fp64;
};
// out (=|+=) scale * in, converting precision and layout.
hipError_t copy_field(int64_t V, int cols, FieldDesc in, FieldDesc out, bool accumulate,
                      double scale, hipStream_t st);

// Per-shift update of Sec. 3 in block form, for the listed shifts j:
//   P_j <- V_i - P_j N_j      (or P_j <- V_i on the first step)
//   X_j[:, l] += P_j M_j[:, l] for the columns l set in colmask[j]
// All blocks column-major with column stride nrows.
struct ShiftArgs {
    int64_t nrows;
    const void *V;              // b columns
    int b, bp, m;
    const void *Pold;           // [s][bp][n]
    void *Pnew;                 // [s][b][n]
    int64_t pstride;            // elements between shifts in the P buffers
    void *X;                    // [s][m][n]
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
