// Small FP64 algebra of DSBlockCG on the device: the m x m quantities of the
// block Lanczos process and of the per-shift root-free Cholesky recurrences.
#pragma once

#include "common.hpp"

namespace dsbcg {

constexpr int kS = 16;       // largest shift count / block width handled by the small kernels
constexpr int kStack = 256;  // largest number of stacked right-hand-side columns

// Matrices are 16 x 16 row-major (leading dimension 16); only the leading
// rows x cols part is meaningful.
struct SmallState {
    zd alpha[256];       // alpha_i  (b x b), hermitised
    zd beta[256];        // beta_i   (b x bp)
    zd betanext[256];    // beta_{i+1} (bnew x b)
    zd R1[256];          // first-pass Cholesky factor of W^H W, kept rows (bnew x b)
    zd C1[256];          // E_K R_KK^{-1}                       (b x bnew)
    zd R2inv[256];       // R2^{-1} of the second CholQR pass (bnew x bnew; I when skipped)
    zd Nv[256];          // V_i^H V_i of the current block as stored (b x b): the Gram of the
                         // basis update when its second pass was skipped, else I
    zd cB[3][256];       // coefficients of the basis update
                         //   V' = W C1 - V_i alpha_i C1 - V_{i-1} beta_i^H C1:
                         //   [0] C1, [1] -alpha_i C1, [2] -beta_i^H C1
    zd rho[kS * kStack]; // R factor of the deflated QR of the stacked right-hand sides,
                         // row r, stacked column c at r * kStack + c  (m1 x M)
    zd coef[4][256];     // scratch coefficient matrices for the block kernels
    zd L[kS][256];       // per shift: Cholesky factor of Delta_{j,i} (lower, b x b)
    zd Z[kS][256];       // per shift: Z_{j,i} (b x m)
    zd N[kS][256];       // per shift: N_{j,i} (bp x b)
    zd M[kS][256];       // per shift: M_{j,i} (b x m)
    zd dM[kS][256];      // per shift: change of M_{j,i} made by vector-wise stopping (b x m)
    double sigma[kS];
    double bnorm[kStack];       // norms of the stacked right-hand-side columns
    int32_t colmap[kS][kS];     // stacked column of right-hand side l of shift j
    double test;         // running estimate of ||T||: max Frobenius norm of alpha_i, beta_i
    int32_t b, bp, m, s;
    int32_t skip_qr2;    // the first CholQR pass is orthogonal enough: no second pass
    int32_t redo;        // the first CholQR pass could not resolve a drop decision: the
                         // step's QR is redone column by column (small_wqr_*)
};

// What the host reads after every block step.
struct StepReport {
    int32_t bnew;
    int32_t flags;       // bit 0: Delta not positive definite, bit 1: second QR pass failed,
                         // bit 2: non-finite input, bit 3: rank above 16, bit 4: the
                         // step's QR must be redone column by column
    int32_t kept[kS];    // pivot columns kept by the deflated QR
    uint32_t colmask[kS];// per shift: columns still being updated
    double est[kS][kS];  // [j][l] estimated relative residual
    double scalar[4];    // [0]: norm of the last CGS remainder, [1]: kept flag of that column
    int32_t stage[kS][kS];  // [j][l] vector-wise stopping: the number r of this step's
                            // Lanczos vectors after which (l, j) stopped (0: did not stop)
    int32_t skip_qr2;    // the second CholQR pass of this step was not run
};

enum { kFlagNotHPD = 1, kFlagQR2 = 2, kFlagNonFinite = 4, kFlagRank = 8, kFlagRedoQR = 16 };

// alpha_i = herm(raw Gram V_i^H W) into the state, and coef[1] = -alpha_i.
hipError_t small_prep_alpha(SmallState *st, const zd *alpha_raw, hipStream_t stream);

// Per-shift coefficients of step i from alpha_i (raw Gram, not yet
// hermitised): Delta_{j,i}, its Cholesky factor, N_{j,i} and M_{j,i}.
hipError_t small_shift_coeffs(SmallState *st, StepReport *rep, const zd *alpha_raw, int first,
                              const int32_t *shift_list, int nact, hipStream_t stream);

// Window of block steps i0+1 .. i0+t.  Within it, per shift j,
//   P_{j,i} = P_{j,i0} Wg_j + sum_u V_{i0+1+u} Wh_{j,u}
//   X_j increment = P_{j,i0} Wfp_j + sum_u V_{i0+1+u} Wf_{j,u}
// (16 x 16 row-major FP64 blocks; rows of Wh_{j,u}, Wf_{j,u} beyond the width
// of V_{i0+1+u} are zero).  Device arrays, allocated by the caller.
constexpr int kWinMax = 128;  // largest window length in block steps
struct WinCoef {
    zd *Wg;          // [kS][256]   b_{i0} x b_i
    zd *Wfp;         // [kS][256]   b_{i0} x m
    zd *Wh;          // [kS][kWinMax][256]
    zd *Wf;          // [kS][kWinMax][256]
    uint32_t *Wmask; // [kS] columns of X_j updated in the window
    int32_t *Wcount; // [kS] window slots holding coefficients of shift j
};
size_t wincoef_bytes();
WinCoef wincoef_at(void *base);

// Window bookkeeping for step i (after small_shift_coeffs): slot t = i - i0 - 1,
// b_{i0} (0 when the window starts at step 1, i.e. there is no stored P),
// current and previous widths, m.
struct WindowStep {
    int t, bp0, b, bp, m;
};
hipError_t small_window_update(const SmallState *st, const StepReport *rep, WinCoef wc, WindowStep ws,
                               const int32_t *shift_list, int nact, hipStream_t stream);
hipError_t small_window_reset(WinCoef wc, hipStream_t stream);

// Coefficient table of the window contraction in the data precision, in the
// lane order of the 16x16x4 matrix-core product (see window_apply):
// table[js][pair][mt][lane], lane = i + 16 k, for output row i of tile mt
// (a real or imaginary part of complex output 8 mt + 0..7: X column if
// < m, else P column - m) and input real index k of the pair (real or
// imaginary part of complex input 2 pair + k / 2: the P_{j,i0} columns
// first, then the window columns).
struct WindowTable {
    int nshift;     // shifts of the window (order of `shifts`)
    int bp0, m, bend;
    int pairs_p;    // ceil(bp0 / 2)
    int ncolv;      // window columns (sum of the widths)
    int npairs;     // pairs_p + ceil(ncolv / 2)
    int nmt;        // 16-column output tiles: ceil(2 (m + bend) / 16)
    int K;          // window slots of this table (a contiguous part of the window)
    int slot0;      // window slot of the first of them
    int wb[kWinMax];// widths of those blocks
};
hipError_t small_window_table(const WinCoef wc, const WindowTable &wt, const int32_t *shifts,
                              const int32_t *pmask, bool fp64, void *table, hipStream_t stream);

// Table of the three-product window contraction (WinArgs.gauss) for a
// window part with no P_{j,i0} inputs (bp0 = 0) and m + bend <= 8:
// table[js2][blk][t][64] for shift pairs js2 < ceil(nshift / 2) and blocks
// of 4 input columns blk < ceil(ncolv / 4), t = 0, 1, 2 (real part,
// imaginary part, their sum); lane order in window_table3_kernel.
hipError_t small_window_table3(const WinCoef wc, const WindowTable &wt, const int32_t *shifts,
                               const int32_t *pmask, bool fp64, void *table, hipStream_t stream);

// Combined table of the partial-fraction window update (rational_window_apply):
// table[pair][mt][lane] in the same lane order, for the outputs 0..m-1 of Y,
// with input pairs [P_{j,i0} of each window shift (ceil(bp0 / 2) pairs each,
// in the order of `shifts`) | window columns].  Entries: c_j Fp_j for the
// P_{j,i0} inputs and sum_j c_j F_{j,u} for the window columns (coef: device
// [kS] real coefficients by shift index).  wt.bend is ignored.
hipError_t small_rational_table(const WinCoef wc, const WindowTable &wt, const int32_t *shifts,
                                const double *coef, bool fp64, void *table, hipStream_t stream);

// First pass of the deflated CholQR of W: Cholesky of G = W^H W with column
// dropping (remainder <= tau_W * ||T||_est); also updates ||T||_est from
// alpha_i and beta_i.  Sets skip_qr2 when the kept columns, scaled to unit
// norm, have a condition number of at most 16 (bounded through the Frobenius
// norms of the scaled factor and its inverse): one CholQR pass then leaves
// their loss of orthogonality at a few hundred units of rounding, and the
// second pass is not run.
//
// The Schur remainder d_k = G_kk - sum |R_rk|^2 carries rounding of a few
// units of G_kk, so a remainder below kResolve * G_kk does not decide a drop
// against a threshold below that level.  Then the kernel sets st->redo and
// the kFlagRedoQR report flag and skips the second pass; small_finish and the
// basis scaling (whose launch takes &st->redo as its skip flag) do nothing,
// and the host redoes the step's QR by classical Gram-Schmidt applied twice
// on the tall-skinny block (small_wqr_*), which resolves a remainder to a
// few units of rounding of ||w_k||.
constexpr double kResolve = 1e-10;
// Smallest drop threshold tau_W of block steps run with FP32 vectors.
constexpr double kTauW32 = 1e-5;
hipError_t small_chol_deflate(SmallState *st, StepReport *rep, const zd *alpha_raw, const zd *G,
                              double tau_W, hipStream_t stream, const zd *Gref = nullptr);

// Gram of the orthogonalised block from the quantities of one pass over
// W' = W - V_{i-1} beta_i^H: with M = V_i^H W' (alpha_i = herm(M) already in
// the state), G' = W'^H W' and N = V_i^H V_i (Nv), the Gram of
// W'' = W' - V_i alpha_i is exactly
//   W''^H W'' = G' - M^H alpha_i - alpha_i^H M + alpha_i^H N alpha_i.
// N is the Gram of V_i as stored, measured when V_i was written: taking it
// for I would feed the basis's departure from orthonormality into the next
// Gram, amplified by about ||alpha||^2 / ||beta||^2 every step.  The rounding
// of the result is of the order of the entries of G', so small_chol_deflate
// takes G' as the reference scale of its resolution rule (Gref).  Writes the
// b x b result to G.
hipError_t small_lanczos_gram(const SmallState *st, const zd *M, const zd *Gp, zd *G, hipStream_t stream);

// Nv = G (the b x b Gram of V_i as stored, e.g. after its rounding to FP32).
hipError_t small_set_nv(SmallState *st, const zd *G, hipStream_t stream);

// cB[0..2] from C1, alpha_i and beta_i (after small_chol_deflate).
hipError_t small_basis_coefs(SmallState *st, hipStream_t stream);

// Column-by-column deflated QR of W (classical Gram-Schmidt applied twice,
// column order, the rule of the initial QR with the absolute threshold
// tau * ||T||_est): small_wqr_begin clears R1; small_wqr_decide stores
// column l's coefficients c1 + c2 on the k kept vectors in R1 and keeps the
// column (new row k, R1[k][l] = ||w||) when ||w|| > tau * ||T||_est, writing
// coef[3] = 1/||w|| and the decision into rep->scalar like small_cgs_decide;
// small_wqr_end records the kept columns, sets beta_{i+1} = R1 (no second
// pass) and clears the redo flag, after which small_finish runs as usual.
hipError_t small_wqr_begin(SmallState *st, hipStream_t stream);
hipError_t small_wqr_decide(SmallState *st, StepReport *rep, const zd *c1, const zd *c2, const zd *nu2,
                            int k, int l, double tau, hipStream_t stream);
struct WqrKept {
    int32_t col[kS];
};
hipError_t small_wqr_end(SmallState *st, StepReport *rep, int nk, WqrKept kept, hipStream_t stream);

// Second pass: R2 from G2 = Q1^H Q1 (Q1 = W'' C1, the basis update as
// stored), R2inv = R2^{-1}, beta_{i+1} = R2 R1, C_j = -beta_{i+1} M_{j,i}
// (= Z_{j,i+1}), estimated residuals and freezing; Nv = G2 when the second
// pass is skipped, else I; rotates b, bp.  Does nothing while st->redo is set.
hipError_t small_finish(SmallState *st, StepReport *rep, const zd *G2, double tol, int freeze,
                        const int32_t *shift_list, int nact, hipStream_t stream);

// Vector-wise stopping granularity (Sec. 3: the iterates advance one Lanczos
// vector at a time, X^(k) = X^(k-1) + p^(k) u^(k) / d^(k)).  Run after
// small_finish (called with freeze = 0) of block step i, width b: for every
// system (l, j) still updated it evaluates the residual estimates of the
// Galerkin iterates on the first K_{i-1} + r basis vectors, r = 1..b, and
// stops the system at the first r whose estimate is <= tol (clearing its
// colmask bit, with est and stage[j][l] = r in the report).  When r < b its
// update of this step is the leading part P_{j,i}[:, 1..r] y_r of the block
// update, and dM_j holds the change of its column of M_{j,i}; otherwise dM_j
// is zero.  Does nothing while st->redo is set.
hipError_t small_vector_stop(SmallState *st, StepReport *rep, double tol, const int32_t *shift_list,
                             int nact, hipStream_t stream);
// Add dM_j into the window coefficients of step i (ws as given to
// small_window_update for that step): Wfp_j += Wg_j dM_j, Wf_{j,u} += Wh_{j,u} dM_j
// (u < t) and Wf_{j,t} += dM_j.  Does nothing while st->redo is set.
hipError_t small_window_correct(const SmallState *st, WinCoef wc, WindowStep ws, const int32_t *shift_list,
                                int nact, hipStream_t stream);

// Initial deflated QR of B, classical Gram-Schmidt twice per column.
// small_bnorms: ||b_l|| for the stacked columns c0 .. c0+cnt-1 from the diagonal of
// their Gram matrix; flags non-finite columns.
hipError_t small_bnorms(SmallState *st, StepReport *rep, const zd *G, int c0, int cnt,
                        hipStream_t stream);
// coef[slot] = -(column 0 of src) for the first k rows.
hipError_t small_neg_column(SmallState *st, int slot, const zd *src, int k, hipStream_t stream);
// Decide on column l: rho[0..k)[l] = c1 + c2; keep if ||w|| > tau_B ||b_l||.
// Writes coef[3] = 1/||w|| and the decision into rep->scalar.
hipError_t small_cgs_decide(SmallState *st, StepReport *rep, const zd *c1, const zd *c2,
                            const zd *nu2, int k, int l, double tau_B, hipStream_t stream);
// Initialise the per-shift state from rho: Z_{j,1} = the columns of rho that
// belong to shift j (per_shift: stacked column j*m + l, else column l for
// every shift), masks and estimates.
hipError_t small_init_shifts(SmallState *st, StepReport *rep, int m1, int m, int s,
                             const double *sigma_host, int freeze, double tol, int per_shift,
                             hipStream_t stream);

}  // namespace dsbcg
