/*
 * dsbcg.h -- C ABI of the MI355X (gfx950) library for the deflated shifted
 * block CG method (DSBlockCG) of Birk & Frommer, "A CG Method for Multiple
 * Right Hand Sides and Multiple Shifts in Lattice QCD Calculations".
 *
 * Problem (Sec. 1, eqs. (1.1) and (1.2)): for m right-hand sides
 * B = [b_1 | ... | b_m] and s real shifts sigma_j, solve
 *
 *        (sigma_j I + A) X_j = B,   j = 1..s,
 *
 * with A = D^H D and D the Wilson-Dirac operator on a periodic 4-d lattice
 * (the paper names "the Wilson fermion matrix"; its conventions are fixed
 * here):
 *
 *   (D psi)(x) = psi(x) - kappa sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                                      + (1 + g_mu) U_mu(x-mu)^H psi(x-mu) ]
 *
 * hermitian gamma matrices in the chiral (DeGrand-Rossi) basis, periodic
 * boundaries, site index x + Lx*(y + Ly*(z + Lz*t)), U_mu(x) on the link
 * x -> x+mu.
 *
 * Memory layouts (C order):
 *   U   complex128 [V][4][3][3]     U[x][mu][a][b] = (U_mu(x))_{ab}
 *   B   complex128 [V][4][3][m]     right-hand side innermost
 *   X   complex128 [s][V][4][3][m]  one block per shift
 * complex128 = two IEEE doubles (re, im), 16-byte aligned.
 *
 * All array pointers are DEVICE pointers (memory of the current HIP device)
 * unless a comment says "host".  The caller owns every array it passes; the
 * handle owns its neighbour geometry and a workspace that grows on demand and
 * is freed by dsbcg_destroy.  Inputs are never modified.  Calls on one handle
 * must not overlap; distinct handles are independent.
 *
 * Every call returns a dsbcg_status; on failure dsbcg_last_error() returns a
 * message for the calling thread.
 */
#ifndef DSBCG_H
#define DSBCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dsbcg_ctx *dsbcg_handle;
typedef void *dsbcg_stream; /* a hipStream_t; NULL = the null stream */

typedef enum {
    DSBCG_OK = 0,
    DSBCG_ERR_ARG = 1,           /* bad sizes, NULL pointer, m or s out of range, tol <= 0,
                                    non-finite sigma or kappa */
    DSBCG_ERR_NOT_HPD = 2,       /* a shifted block Delta_{j,i} lost positive definiteness:
                                    sigma_j I + A is not hpd (or B, U hold NaN/Inf) */
    DSBCG_ERR_NOT_CONVERGED = 3, /* max_iters reached; X holds the current iterates */
    DSBCG_ERR_HIP = 4,           /* HIP runtime error */
    DSBCG_ERR_OOM = 5            /* device allocation failed */
} dsbcg_status;

typedef enum {
    DSBCG_FP64 = 0,          /* every vector operation in FP64 */
    DSBCG_FP32_RELIABLE = 1  /* FP64 vectors until the estimates reach opts.switch_at, then
                                FP32 stencil and block updates; FP64 small algebra, FP64
                                solution accumulation, FP64 true residuals of every system at
                                the end and re-solves of the shifts that miss tol */
} dsbcg_precision;

/* Largest supported number of right-hand sides and of shifts. */
#define DSBCG_MAX_RHS 16
#define DSBCG_MAX_SHIFTS 16

typedef struct {
    int32_t precision;    /* dsbcg_precision */
    int32_t max_iters;    /* block-step limit of the main phase (default 10000) */
    int32_t fixed_iters;  /* > 0: run exactly this many block steps, no convergence stop */
    int32_t ru_interval;  /* FP32 form: the contribution of the FP32 Lanczos blocks is added
                             into the FP64 solution at least every this many block steps and at
                             the end (default 50) */
    double tau_B;         /* initial deflation of B: drop column l when its remainder is
                             <= tau_B * ||b_l|| (default 0.1 * tol) */
    double tau_W;         /* in-iteration deflation: drop a new basis column whose remainder is
                             <= tau_W * ||T||_est, ||T||_est the running maximum of the
                             Frobenius norms of the alpha_i and beta_i (default 1e-12; steps
                             run with FP32 vectors use max(tau_W, 1e-5)).  The remainder is
                             the Schur complement of the Cholesky factorisation of W^H W;
                             where that cannot resolve the decision (a remainder below 1e-10
                             times the column's squared norm while the threshold lies below
                             that level) the step's QR is redone by classical Gram-Schmidt
                             applied twice, column by column, as for B */
    int32_t refine;       /* 1: after the main phase, re-solve the shifts whose true residual
                             misses tol, (sigma_j + A) E = R_j, X_j += E (default 1); in the FP32
                             form the first round of re-solves runs with FP32 vectors, a second
                             round (if needed) in FP64 */
    int32_t freeze;       /* 1: stop updating a system once its estimate reaches tol (default 1) */
    int32_t window;       /* per-shift update window: the Lanczos blocks of up to `window`
                             block steps are kept and X_j (and P_j, if the iteration goes on)
                             are formed from them once per window.  0: the longest window
                             whose blocks fit in three quarters of the free device memory less
                             4 GiB, at most 128;
                             1: every step.  The result is the same up to rounding */
    double switch_at;     /* FP32 form: the iteration runs in FP64 until every active estimated
                             relative residual is <= switch_at, then continues the same
                             recurrences with FP32 vectors (default min(1e-2, 1e5 * tol)) */
    int32_t keep_workspace; /* 1 (default): the handle keeps the device workspace of a solve
                             (the kept Lanczos blocks, allocated as the windows take them; P_j,
                             allocated only when a window forms them; the column-major
                             iterates and right-hand sides) for the next call, which then
                             allocates nothing it already holds; free it with
                             dsbcg_release_workspace.  0: the solve frees it before it returns
                             (the staged links stay).  Allocating the workspace of the
                             32^3 x 64, m = 8, s = 10 solve costs seconds, against 0.42 s
                             for the solve itself */
    int32_t vector_stop;  /* 1: stopping granularity of one Lanczos vector (Sec. 3: the iterates
                             advance one basis vector at a time, X^(k) = X^(k-1) + p^(k) u^(k) /
                             d^(k)): inside every block step the residual estimates of the
                             Galerkin iterates on the first K + r basis vectors (K before the
                             block, r = 1..b) are formed from the block's small matrices, and a
                             system stops at the first r whose estimate is <= tol, keeping that
                             iterate.  Needs freeze = 1.  The block step still applies A to all
                             its b vectors, so the saving is in the iterate, not in time; see
                             dsbcg_stats.mvms_vector.  0 (default): systems stop at block
                             boundaries */
} dsbcg_opts;

typedef struct {
    int32_t block_iters;      /* block steps of the main phase */
    int32_t rank0;            /* width of the first Lanczos block after deflating B */
    int32_t deflations;       /* columns dropped during the iteration */
    int32_t reliable_updates; /* FP32 form: windows of FP32 blocks added into the FP64
                                 solution */
    int32_t refine_iters;     /* block steps spent in refinement solves */
    int32_t final_width;      /* width of the last Lanczos block */
    int32_t switch_iter;      /* FP32 form: first block step run with FP32 vectors (0: none) */
    int32_t qr2_skipped;      /* block steps whose second CholQR pass was not needed (the
                                 unit-norm kept columns had condition number <= 16) */
    double main_relres_max;   /* largest FP64 true relative residual after the main phase,
                                 before any re-solve (0 when true residuals were not formed;
                                 -1 in the FP64 partial-fraction form) */
    int64_t mvms;             /* applications of A to one vector by the method: sum of the
                                 block widths of the main phase and of refinement solves */
    double *est_relres;       /* host [s*m] (index j*m + l) or NULL: last estimated
                                 relative residuals */
    double *true_relres;      /* host [s*m] or NULL: FP64 true relative residuals
                                 ||b_l - (sigma_j + A) x_{l,j}|| / ||b_l|| at return */
    int32_t *widths;          /* host [widths_len] or NULL: width m_i of the Lanczos block of
                                 main-phase step i at widths[i-1] (0 past the last step; not
                                 filled when dsbcg_solve_multi falls back to one solve per
                                 shift) */
    int32_t widths_len;
    int32_t qr_redone;        /* block steps whose deflated QR was redone column by column
                                 (see dsbcg_opts.tau_W) */
    int64_t mvms_vector;      /* main phase: the number of Lanczos vectors through the stage at
                                 which the last system stopped, i.e. the applications of A the
                                 vector-wise process of Sec. 3 needs (every vector of the run
                                 when some system never stopped); equals the block count of the
                                 stopping step's end unless opts.vector_stop = 1 */
    int32_t *frozen_at;       /* host [s*m] (index j*m + l) or NULL: main phase, the number of
                                 Lanczos vectors through the stage at which (l, j) stopped (0:
                                 it never stopped, or its column of B is zero) */
    double *est_history;      /* host [widths_len] or NULL: residual history of the main phase,
                                 the largest estimated relative residual over the systems still
                                 updated after step i at est_history[i-1] (0 past the last step) */
} dsbcg_stats;

/* Fill opts with the defaults listed above. */
void dsbcg_default_opts(dsbcg_opts *opts);

/* Create a handle for a lattice L = {Lx, Ly, Lz, Lt} (host array; each
 * extent >= 2, volume < 2^31 / 12).  Binds the handle to the current device. */
int dsbcg_create(const int32_t *L, dsbcg_handle *out);

/* Release the handle and its workspace (NULL is ignored). */
void dsbcg_destroy(dsbcg_handle h);

/* Free the device workspace a handle holds (after solves with
 * opts.keep_workspace = 1, or the staging buffers of dsbcg_apply_A), keeping
 * the staged links.  Synchronises the device. */
int dsbcg_release_workspace(dsbcg_handle h);

/* Export the neighbour table the kernels use: host_out[V][8] receives the
 * sites x+x^, x-x^, x+y^, x-y^, x+z^, x-z^, x+t^, x-t^ (host array, caller
 * allocated).  Synchronous. */
int dsbcg_neighbors(dsbcg_handle h, int32_t *host_out);

/* Stage the links once (Sec. 1: the gauge links U_mu(x) are the coefficients
 * of the Wilson matrix): U is checked for NaN/Inf (DSBCG_ERR_NOT_HPD, as in
 * dsbcg_solve) and converted to the FP64 and FP32 structure-of-arrays copies
 * the kernels read, held by the handle (0.86 KB per site).  Afterwards every
 * call below that takes U accepts U = NULL and uses the staged copy without
 * converting it again; a call with U != NULL converts that U into the same
 * buffers and the staged copy is gone.  Returns with `stream` synchronised. */
int dsbcg_stage_links(dsbcg_handle h, const void *U, dsbcg_stream stream);

/* Y = A X = D^H (D X) for m columns (1 <= m <= DSBCG_MAX_RHS).
 * U, X, Y: device, layouts above (X, Y are [V][4][3][m]); Y must not alias X;
 * U may be NULL after dsbcg_stage_links.
 * precision DSBCG_FP64 computes in FP64; DSBCG_FP32_RELIABLE rounds U and X
 * to FP32, applies the FP32 stencil and writes the FP32 result widened to
 * FP64.  Asynchronous on `stream`. */
int dsbcg_apply_A(dsbcg_handle h, const void *U, double kappa, const void *X, void *Y,
                  int32_t m, int32_t precision, dsbcg_stream stream);

/* dsbcg_apply_A without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, results (bit for bit) and errors as
 * dsbcg_apply_A; U may be NULL after dsbcg_stage_links.  The column-major
 * staging of X, the intermediate D X and, when U is given, the converted
 * links live in one fixed workspace per device of 128 MiB (held by every GPU
 * the library runs on until the process ends; the second pass writes Y in
 * the caller's layout directly), so a call needs
 *     V * 36 * e  (only when U != NULL)  +  2 * 12 * V * m * e  bytes,
 * e = 16 (FP64) or 8 (FP32), each part rounded up to 256 bytes; a larger call
 * returns DSBCG_ERR_ARG and leaves Y untouched.  The handle must belong to
 * the current device.  Every call on one GPU uses the same workspace: calls
 * that overlap on one GPU (other streams or threads) race.  Asynchronous on
 * `stream`; no hipMalloc, hipFree or allocating library routine is called. */
int dsbcg_apply_A_noalloc(dsbcg_handle h, const void *U, double kappa, const void *X, void *Y,
                          int32_t m, int32_t precision, dsbcg_stream stream);

/* Y = D X (dagger = 0) or D^H X (dagger = 1), FP64, same layouts as
 * dsbcg_apply_A (U may be NULL after dsbcg_stage_links).  Asynchronous on
 * `stream`. */
int dsbcg_apply_D(dsbcg_handle h, const void *U, double kappa, const void *X, void *Y,
                  int32_t m, int32_t dagger, dsbcg_stream stream);

/* Solve (sigma_j I + A) X_j = B for j = 0..s-1 with DSBlockCG (Sec. 3).
 * U, B: device inputs (U may be NULL after dsbcg_stage_links; this and the
 * other solve entry points then skip the link check and conversion);
 * sigma: HOST array of s real shifts with sigma_j I + A
 * hpd; X: device output [s][V][4][3][m], fully written.  tol: target relative
 * residual ||b_l - (sigma_j + A) x_{l,j}|| <= tol ||b_l|| for every (l, j)
 * (Sec. 4).  opts may be NULL (defaults); stats may be NULL.
 * Returns with `stream` synchronised (the iteration takes host decisions
 * after every block step).  Zero columns of B give zero columns of X. */
int dsbcg_solve(dsbcg_handle h, const void *U, double kappa, const void *B, int32_t m,
                const double *sigma, int32_t s, double tol, const dsbcg_opts *opts,
                void *X, dsbcg_stats *stats, dsbcg_stream stream);

/* Partial-fraction form (Sec. 1: the rational approximation of a matrix power
 * that the rational hybrid Monte Carlo algorithm needs, written as a partial
 * fraction expansion, is what gives rise to the shifted systems):
 *
 *     Y = c0 B + sum_j coef_j (sigma_j I + A)^{-1} B
 *
 * coef: HOST array of s real coefficients; c0 a real scalar; Y: device output
 * [V][4][3][m], fully written, must not alias B.  Other arguments as
 * dsbcg_solve; every system (l, j) is iterated to the same tol.
 *   DSBCG_FP64: the per-shift X_j are never formed.  The window contraction
 *     accumulates sum_j coef_j X_j directly into Y (one output block instead
 *     of s), and no s*V*12*m workspace is held.  Convergence is decided by the
 *     estimated residuals of the method (Sec. 3): stats->true_relres is filled
 *     with -1 (not formed) and main_relres_max is -1.
 *   DSBCG_FP32_RELIABLE: the checked solve of dsbcg_solve (FP64 true
 *     residuals, re-solves of shifts that miss tol) into a workspace of
 *     s*V*12*m complex128, then the sum.
 * A frozen or converged system contributes its final iterate.  Returns with
 * `stream` synchronised; errors as dsbcg_solve (ERR_NOT_CONVERGED leaves the
 * sum of the current iterates in Y). */
int dsbcg_solve_rational(dsbcg_handle h, const void *U, double kappa, const void *B, int32_t m,
                         const double *sigma, const double *coef, int32_t s, double c0, double tol,
                         const dsbcg_opts *opts, void *Y, dsbcg_stats *stats, dsbcg_stream stream);

/* Solve (sigma_j I + A) X_j = B_j for j = 0..s-1, one right-hand-side block
 * per shift: B is [s][V][4][3][m] (device).  The blocks are stacked and
 * deflated together (deflated QR of [B_0 | ... | B_{s-1}]) and ONE DSBlockCG
 * run over that common basis serves every shift, each with its own initial
 * coefficients (the block form of the paper's method with Z_{j,1} = the
 * coordinates of B_j).  When the blocks span more than 16 directions the call
 * falls back to one block solve per shift.  This is the adjoint solve of the
 * differentiation form: Lambda_j = (sigma_j + A)^{-1} dL/dX_j.  Other
 * arguments, results and errors as dsbcg_solve. */
int dsbcg_solve_multi(dsbcg_handle h, const void *U, double kappa, const void *B, int32_t m,
                      const double *sigma, int32_t s, double tol, const dsbcg_opts *opts,
                      void *X, dsbcg_stats *stats, dsbcg_stream stream);

/* Backward of X_j = (sigma_j I + D^H D)^{-1} B (U may be NULL after
 * dsbcg_stage_links) given X_j and the adjoint
 * solutions Lambda_j = (sigma_j I + A)^{-1} G_j, G_j = dL/dRe X_j + i dL/dIm X_j
 * (both [s][V][4][3][m], device).  Since sigma_j I + A is hermitian,
 *   dL/dB       = sum_j Lambda_j                         (dB: device [V][4][3][m])
 *   dL/dsigma_j = -Re <Lambda_j, X_j>                     (dsigma: HOST [s])
 *   dL/dU       = -sum_j [ dRe<D X_j, D Lambda_j> + dRe<D Lambda_j, D X_j> ]/dU
 * (dU: device [V][4][3][3], convention dRe + i dIm, link-derivative stencil of
 * dsbcg_link_grad).  Each output pointer may be NULL to skip it.  Synchronises
 * `stream` when dsigma is requested. */
int dsbcg_grad(dsbcg_handle h, const void *U, double kappa, const double *sigma, int32_t s,
               int32_t m, const void *X, const void *Lam, void *dU, void *dB, double *dsigma,
               dsbcg_stream stream);

/* Link derivative of f(U) = sum_k Re <Phi_k, D[U] Psi_k> summed over the
 * nvec = s*m columns of Phi and Psi ([V][4][3][nvec], device), in the
 * convention dU = df/dRe U + i df/dIm U:
 *
 *   dU_mu(x) = -kappa sum_{spin, k} [ ((1 - g_mu) Phi(x)) Psi(x+mu)^H
 *                                   + Psi(x) ((1 + g_mu) Phi(x+mu))^H ]
 *
 * dU: device [V][4][3][3], overwritten.  FP64.  Asynchronous on `stream`. */
int dsbcg_link_grad(dsbcg_handle h, double kappa, const void *Phi, const void *Psi,
                    int32_t nvec, void *dU, dsbcg_stream stream);

/* Kernel timing.  While enabled, every kernel the calls on h launch is
 * bracketed by two HIP events on the call's stream (this adds a few
 * microseconds per launch); durations and algorithmic bytes (the data each
 * kernel must read and write, not cache traffic) accumulate per kernel class.
 * dsbcg_profile_enable resets the totals.  Classes (dsbcg_profile_name):
 * 0/1 Wilson stencil pass D or D^H in FP64/FP32, 2/3 block Gram / combination
 * kernels in FP64/FP32, 4/5 windowed per-shift P_j / X_j update in FP64/FP32,
 * 6 small FP64 algebra and Gram reductions, 7 conversions, 8 link derivative.
 * dsbcg_profile_read waits for the recorded events; any pointer may be NULL. */
int dsbcg_profile_enable(dsbcg_handle h, int32_t enable);
int dsbcg_profile_read(dsbcg_handle h, int32_t kclass, double *ms, int64_t *launches,
                       double *bytes);
/* Time only the classes whose bit is set in class_mask (bit k: class k;
 * 0xffffffff, the default, times every class).  Launches of other classes
 * run without events, so that one class can be timed inside a measured
 * region at the cost of its own launches only.  The mask stays until the
 * next call; dsbcg_profile_enable leaves it as it is. */
int dsbcg_profile_select(dsbcg_handle h, uint32_t class_mask);
/* Name of a kernel class, NULL past the last one. */
const char *dsbcg_profile_name(int32_t kclass);

/* Message of the last failed call on this thread ("" if none). */
const char *dsbcg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DSBCG_H */
