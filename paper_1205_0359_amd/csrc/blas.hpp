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
constexpr int kPartialStride = 512;  // partial Gram entries per workgroup (two 16 x 16 blocks)

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
    int gram;                // 0: none, 1: partial out^H out, 2: partial L^H out,
                             // 3: diagonal of out^H out only, 4: both L^H out (partial
                             // entries 0..255 of the workgroup) and out^H out (256..511)
    const void *L;
    int64_t csl;
    int bl;
    zd *partials;            // [nwg][kPartialStride] FP64 partial Gram matrices (16 x 16 each)
    int64_t rows_per_wg;
    const int32_t *skip;     // device flag or NULL: when set the launch does nothing
};

// Launch the combination / Gram kernel; *nwg receives the workgroup count
// whose partials must be reduced (at most max_wg).
hipError_t ts_run(bool fp64, TsArgs a, int max_wg, int *nwg, hipStream_t st);

// out[e] = sum_w partials[w][off + e] for e < nelem, summed in a fixed order.
hipError_t reduce_partials(const zd *partials, int nwg, int nelem, zd *out, hipStream_t st, int off = 0);

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

// Window update of the per-shift iterates over the block steps of a window:
//   X_j += P_{j,i0} Fp_j + sum_u V_u F_{j,u}          (columns in xmask[j])
//   P_{j,end} = P_{j,i0} G_j + sum_u V_u H_{j,u}      (shifts with pmask set)
// as one matrix-core contraction per shift: the inputs [P_{j,i0} | V_window]
// (complex columns taken in pairs) times the coefficient table built by
// small_window_table.  The window columns are shared by all shifts and are
// staged chunk by chunk in LDS; X is FP64 in both precisions.
struct WinArgs {
    int64_t nrows;
    int ncolv;                  // window columns (sum of the block widths)
    const void *const *colptr;  // device array [ncolv]: first element of each window column
    int bp0;                    // width of P_{j,i0} (0: no P term)
    const void *Pold;
    void *Pnew;
    int bend;                   // width of P_{j,end}
    int64_t pstride;            // elements between shifts in the P buffers
    int m;
    zd *X;                      // [s][m][nrows] FP64
    int64_t xstride;
    const void *table;          // [nshift][npairs][nmt][64] in the data precision
    int npairs, pairs_p, nmt;
    const int32_t *shifts;      // device [nshift]: shift of each window slot
    int nshift;                 // <= 16
    const uint32_t *xmask;      // [s] columns of X_j to update
    const int32_t *pmask;       // [s] nonzero: write P_{j,end}
    int xinit;                  // nonzero: X_j of the window's shifts is overwritten (every
                                // column; the coefficients of columns never updated are zero)
    // Optional second part of the same window in FP32 (a window that spans the
    // switch to FP32 vectors, FP64 first part): its columns and table (no
    // P_{j,i0} pairs) are contracted in FP32 and the two parts are added
    // before X_j and P_{j,end} are written; P_{j,end} then goes to Pnew2 in
    // FP32.  ncolv2 = 0: no second part.
    int ncolv2;
    const void *const *colptr2;
    const void *table2;         // [nshift][npairs2][nmt][64] FP32
    int npairs2;                // ceil(ncolv2 / 2)
    void *Pnew2;                // FP32 P buffer, shift j at j * pstride
    // Optional (nullptr: none): the window's shifts' X_j, every one of the m
    // columns, also stored in the caller's layout [s][V][4][3][m]
    // (complex128, V = nrows / 12, shift j at j * nrows * m).
    zd *Xapi;
    // Nonzero: three real products per complex product (window3_kernel);
    // table then comes from small_window_table3 (table2, the FP32 part, still
    // from small_window_table), and the window has no P_{j,i0} inputs
    // (bp0 = 0) and m + bend <= 8 (nmt = 1).
    int gauss;
};
hipError_t window_apply(bool fp64, const WinArgs &a, hipStream_t st);

// Window update of the partial-fraction sum Y = c0 B + sum_j c_j X_j, the
// per-shift iterates never being formed:
//   Y += sum_j c_j (P_{j,i0} Fp_j + sum_u V_u F_{j,u})
// as ONE matrix-core contraction of [P_{j_1,i0} | ... | P_{j_s,i0} | V_window]
// with the combined table of small_rational_table.  No input is shared
// between waves, so each wave owns its rows and streams its inputs.
struct RatArgs {
    int64_t nrows;
    int ncolv;                  // window columns
    const void *const *colptr;  // device array [ncolv]
    int bp0;                    // width of each P_{j,i0} (0: no P term)
    const void *Pold;           // P buffer, shift j at j * pstride
    int64_t pstride;
    const int32_t *shifts;      // device [nshift]
    int nshift;                 // <= 16
    int m;                      // columns of Y
    zd *Y;                      // [m][nrows] FP64, accumulated
    const void *table;          // [npairs][nmt][64] in the data precision
    int pairs_p;                // ceil(bp0 / 2) pairs per shift
    int npairs;                 // nshift * pairs_p + ceil(ncolv / 2)
    int nmt;                    // ceil(m / 8)
};
hipError_t rational_window_apply(bool fp64, const RatArgs &a, hipStream_t st);

// Checks a field for NaN/Inf: sets *flag (device int) to 1 if any is found.
hipError_t find_nonfinite(const double *data, int64_t count, int32_t *flag, hipStream_t st);

}  // namespace dsbcg
