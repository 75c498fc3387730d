// DSBlockCG driver and C ABI (see include/dsbcg.h).
//
// The block step (Sec. 3 of the paper, block form):
//   W = A V_i                                   Wilson stencil D, then D^H
//   alpha_i = herm(V_i^H (W - V_{i-1} beta_i^H)) Gram kernel
//   per shift: Delta, N, M (small FP64 kernel); P_j, X_j updates (one kernel)
//   W <- W - V_{i-1} beta_i^H - V_i alpha_i, G1 = W^H W
//   deflated Cholesky QR of W, twice -> V_{i+1}, beta_{i+1}
//   residual coefficients C_j = Z_{j,i+1}, estimates, freezing
// The host reads one small report per step (new block width, masks,
// estimates) and decides whether to continue.
//
// Internal layouts: every n x b block is column-major (column stride n =
// 12 V, row c * V + x); links are structure of arrays [4][9][V].  The caller's
// arrays use the site-major layouts of the header and are converted at entry
// and exit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dsbcg.h"
#include "blas.hpp"
#include "grad.hpp"
#include "noalloc.hpp"
#include "small.hpp"
#include "stencil.hpp"

using namespace dsbcg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            if (e_ == hipErrorOutOfMemory)                                                 \
                return fail(DSBCG_ERR_OOM, std::string("out of device memory at ") + #expr); \
            return fail(DSBCG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
        }                                                                                  \
    } while (0)

#define CHK(expr)                          \
    do {                                   \
        int rc_ = (expr);                  \
        if (rc_ != DSBCG_OK) return rc_;   \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

enum ProfClass {
    kProfStencil = 0,   // one Wilson D or D^H pass, FP64 (FP32: + 1)
    kProfBlock = 2,     // tall-skinny combination / Gram kernels of the block step
    kProfShift = 4,     // windowed per-shift P_j / X_j update
    kProfSmall = 6,     // small FP64 algebra and Gram reductions
    kProfConvert,       // layout conversions, widening, accumulation
    kProfGrad,          // link-derivative stencil
    kProfClasses
};
const char *const kProfNames[kProfClasses] = {
    "wilson_stencil.f64", "wilson_stencil.f32", "block_gram_update.f64", "block_gram_update.f32",
    "shift_update.f64",   "shift_update.f32",   "small_algebra",         "convert",
    "link_grad"};
// class of a kernel family in the given data precision
inline int prof_cls(int family, bool fp64) { return family + (fp64 ? 0 : 1); }

struct ProfRec {
    int cls;
    hipEvent_t a, b;
    double bytes;
};

}  // namespace

struct dsbcg_ctx {
    Geom g{};
    int device = 0;
    // kernel timing (dsbcg_profile_enable); prof_mask: classes timed
    // (dsbcg_profile_select)
    bool prof = false;
    uint32_t prof_mask = 0xffffffffu;
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    double prof_ms[kProfClasses] = {};
    double prof_bytes[kProfClasses] = {};
    int64_t prof_launches[kProfClasses] = {};
    // workspace
    DevBuf Ul64, Ul32;                                   // structure-of-arrays links
    DevBuf V0, T, W, P[2], X;                            // FP64 iteration (V0: V_1)
    DevBuf T32, W32, P32[2];                             // FP32 iteration
    DevBuf wcoef, wtable, colptr;                        // window coefficients, MFMA table, columns
    DevBuf Bint, Q, wbuf;                                // deflated QR of B
    DevBuf R0, R1, R2, R3, Rres, Xref;                   // true residuals, refinement
    DevBuf Xin, Yout;                                    // dsbcg_apply_* conversions
    DevBuf Ycm, ycoef, Xrat;                             // partial-fraction form
    DevBuf rpart;                                        // true-residual partial norms
    DevBuf partials, red, list, wlist, st, rep;
    std::vector<DevBuf> Vring, Vring32;                  // window rings of Lanczos blocks
    StepReport *rep_host = nullptr;
    int32_t *list_host = nullptr;
    bool links_staged = false;  // Ul64 and Ul32 hold the links of dsbcg_stage_links
    int nwg_max = 2048;

    ~dsbcg_ctx() {
        DevBuf *all[] = {&Ul64, &Ul32, &V0,  &T,   &W,    &P[0], &P[1], &X,
                         &T32, &W32, &P32[0], &P32[1], &wcoef, &wtable, &colptr,
                         &Bint, &Q,    &wbuf, &R0,   &R1,   &R2,  &R3,   &Rres, &Xref, &Xin,
                         &Yout, &Ycm, &ycoef, &Xrat, &rpart, &partials, &red, &list, &wlist, &st, &rep};
        for (DevBuf *b : all)
            if (b->p) (void)hipFree(b->p);
        for (auto &b : Vring)
            if (b.p) (void)hipFree(b.p);
        for (auto &b : Vring32)
            if (b.p) (void)hipFree(b.p);
        if (rep_host) (void)hipHostFree(rep_host);
        if (list_host) (void)hipHostFree(list_host);
        for (auto &r : prof_pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : prof_pool) (void)hipEventDestroy(e);
    }
};

namespace {

int ensure(DevBuf &b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return DSBCG_OK;
    if (b.p) {
        HIPCHK(hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(DSBCG_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    b.bytes = bytes;
    return DSBCG_OK;
}

// ---- kernel timing: each profiled launch is bracketed by two events ----
hipError_t prof_event(dsbcg_ctx *h, hipEvent_t *e) {
    if (!h->prof_pool.empty()) {
        *e = h->prof_pool.back();
        h->prof_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

struct ProfToken {
    bool on = false;
    hipEvent_t a = nullptr;
};

// whether launches of class cls are timed
inline bool prof_on(const dsbcg_ctx *h, int cls) { return h->prof && ((h->prof_mask >> cls) & 1u); }

ProfToken prof_begin(dsbcg_ctx *h, hipStream_t st, int cls) {
    ProfToken t;
    if (!prof_on(h, cls)) return t;
    if (prof_event(h, &t.a) != hipSuccess) return t;
    if (hipEventRecord(t.a, st) != hipSuccess) return t;
    t.on = true;
    return t;
}

hipError_t prof_end(dsbcg_ctx *h, const ProfToken &t, int cls, double bytes, hipStream_t st) {
    if (!t.on) return hipSuccess;
    hipEvent_t b;
    hipError_t e = prof_event(h, &b);
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, st);
    if (e != hipSuccess) return e;
    h->prof_pending.push_back({cls, t.a, b, bytes});
    return hipSuccess;
}

// Accumulate the finished records (waits for their events).
hipError_t prof_flush(dsbcg_ctx *h) {
    for (auto &r : h->prof_pending) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return e;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return e;
        h->prof_ms[r.cls] += ms;
        h->prof_bytes[r.cls] += r.bytes;
        h->prof_launches[r.cls] += 1;
        h->prof_pool.push_back(r.a);
        h->prof_pool.push_back(r.b);
    }
    h->prof_pending.clear();
    return hipSuccess;
}

#define PROF_LAUNCH(h, cls, bytes, st, expr)                  \
    do {                                                      \
        ProfToken tok_ = prof_begin((h), (st), (cls));        \
        HIPCHK(expr);                                         \
        HIPCHK(prof_end((h), tok_, (cls), (bytes), (st)));    \
    } while (0)

// algorithmic bytes of one Wilson pass on nb columns: read nb spinors and
// the links, write nb spinors
double stencil_bytes(const Geom &g, int nb, size_t esz) {
    return (double)g.V * (2.0 * 12 * nb + 36.0) * (double)esz;
}

double copy_bytes(int64_t V, int cols, size_t in_esz, size_t out_esz, bool accumulate) {
    return (double)V * 12 * cols * ((double)in_esz + (accumulate ? 2.0 : 1.0) * (double)out_esz);
}

// The window rings are sized from the free device memory by each solve and
// kept between solves; a later solve that needs more per-shift memory (more
// shifts, wider blocks) releases them first and sizes them again.
void release_rings(dsbcg_ctx *h) {
    for (auto &b : h->Vring)
        if (b.p) {
            (void)hipFree(b.p);
            b.p = nullptr;
            b.bytes = 0;
        }
    for (auto &b : h->Vring32)
        if (b.p) {
            (void)hipFree(b.p);
            b.p = nullptr;
            b.bytes = 0;
        }
}

// Every device buffer of the handle except the staged links, the small
// algebra state and the partial sums (dsbcg_release_workspace, and the end of
// a solve without opts.keep_workspace).
void release_workspace(dsbcg_ctx *h) {
    release_rings(h);
    DevBuf *big[] = {&h->V0, &h->T, &h->W, &h->P[0], &h->P[1], &h->X, &h->T32, &h->W32, &h->P32[0],
                     &h->P32[1], &h->Bint, &h->Q, &h->wbuf, &h->R0, &h->R1, &h->R2, &h->R3, &h->Rres,
                     &h->Xref, &h->Xin, &h->Yout, &h->Ycm, &h->Xrat, &h->rpart, &h->wtable, &h->colptr};
    for (DevBuf *b : big)
        if (b->p) {
            (void)hipFree(b->p);
            b->p = nullptr;
            b->bytes = 0;
        }
}

// ensure() for per-solve workspace: on a failed allocation the window rings
// are released and the allocation is tried once more.
int ensure_ws(dsbcg_ctx *h, DevBuf &b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return DSBCG_OK;
    if (ensure(b, bytes) == DSBCG_OK) return DSBCG_OK;
    release_rings(h);
    return ensure(b, bytes);
}

int ensure_common(dsbcg_ctx *h) {
    CHK(ensure(h->partials, (size_t)h->nwg_max * kPartialStride * sizeof(zd)));
    CHK(ensure(h->red, 8 * 256 * sizeof(zd)));
    CHK(ensure(h->list, 64 * sizeof(int32_t)));
    CHK(ensure(h->st, sizeof(SmallState)));
    CHK(ensure(h->rep, sizeof(StepReport)));
    if (!h->rep_host) HIPCHK(hipHostMalloc((void **)&h->rep_host, sizeof(StepReport), 0));
    if (!h->list_host) HIPCHK(hipHostMalloc((void **)&h->list_host, 128 * sizeof(int32_t), 0));
    return DSBCG_OK;
}

zd *red_slot(dsbcg_ctx *h, int k) { return (zd *)h->red.p + 256 * k; }

FieldDesc cm(const void *p, int64_t n, bool fp64) { return FieldDesc{const_cast<void *>(p), kCM, n, 0, fp64}; }
FieldDesc api(const void *p, int64_t ld, int col0 = 0) {
    return FieldDesc{const_cast<void *>(p), kApi, ld, col0, true};
}

int copy(dsbcg_ctx *h, int cols, FieldDesc in, FieldDesc out, bool accumulate, hipStream_t st) {
    if (cols <= 0) return DSBCG_OK;
    PROF_LAUNCH(h, kProfConvert,
                copy_bytes(h->g.V, cols, in.fp64 ? 16 : 8, out.fp64 ? 16 : 8, accumulate), st,
                copy_field(h->g.V, cols, in, out, accumulate, 1.0, st));
    return DSBCG_OK;
}

// Tall-skinny combination / Gram launches on column-major blocks.
struct Ts {
    dsbcg_ctx *h;
    bool fp64;
    hipStream_t st;
    int64_t nrows;

    int run(TsArgs a, int *nwg_out) {
        a.nrows = nrows;
        a.partials = (zd *)h->partials.p;
        double per_row = 0;
        for (int k = 0; k < a.K; ++k) per_row += a.bx[k];
        if (a.out) per_row += a.bout;
        if (a.gram == 2 || a.gram == 4) per_row += a.bl;
        const double bytes = per_row * (double)nrows * (fp64 ? sizeof(zd) : sizeof(zf));
        int nwg = 0;
        PROF_LAUNCH(h, prof_cls(kProfBlock, fp64), bytes, st, ts_run(fp64, a, h->nwg_max, &nwg, st));
        if (nwg_out) *nwg_out = nwg;
        return DSBCG_OK;
    }
    // run + reduce of rows p < rows_used into red slot k (gram 4: L^H out
    // into slot k, out^H out into slot k + 1)
    int run_reduce(TsArgs a, int rows_used, int k) {
        int nwg = 0;
        CHK(run(a, &nwg));
        if (rows_used > 0) {
            PROF_LAUNCH(h, kProfSmall, 0.0, st,
                        reduce_partials((zd *)h->partials.p, nwg, rows_used * 16, red_slot(h, k), st));
            if (a.gram == 4)
                PROF_LAUNCH(h, kProfSmall, 0.0, st,
                            reduce_partials((zd *)h->partials.p, nwg, rows_used * 16, red_slot(h, k + 1), st,
                                            256));
        }
        return DSBCG_OK;
    }
};

TsArgs ts_args(int64_t n) {
    TsArgs a;
    memset(&a, 0, sizeof(a));
    for (int k = 0; k < 3; ++k) a.cs[k] = n;
    a.cso = n;
    a.csl = n;
    return a;
}

SmallState *stp(dsbcg_ctx *h) { return (SmallState *)h->st.p; }
StepReport *repp(dsbcg_ctx *h) { return (StepReport *)h->rep.p; }
const zd *coef_slot(dsbcg_ctx *h, int k) { return stp(h)->coef[k]; }

int read_report(dsbcg_ctx *h, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(h->rep_host, h->rep.p, sizeof(StepReport), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h->prof_pending.size() > 4096) HIPCHK(prof_flush(h));
    return DSBCG_OK;
}

int validate_geom(const int32_t *L) {
    if (!L) return fail(DSBCG_ERR_ARG, "L is NULL");
    int64_t V = 1;
    for (int d = 0; d < 4; ++d) {
        if (L[d] < 2) return fail(DSBCG_ERR_ARG, "every lattice extent must be >= 2");
        V *= L[d];
    }
    if (V * 12 >= (int64_t)1 << 31) return fail(DSBCG_ERR_ARG, "lattice volume too large");
    return DSBCG_OK;
}

// Y = D X or D^H X on b column-major columns; with Yapi the result goes to
// the caller's layout [V][4][3][b] (complex128) instead of Y.
int stencil(dsbcg_ctx *h, bool fp64, const void *Ul, double kappa, const void *X, void *Y, int b,
            bool dagger, hipStream_t st, void *Yapi = nullptr) {
    const size_t esz = fp64 ? sizeof(zd) : sizeof(zf);
    const size_t col = (size_t)12 * h->g.V * esz;  // bytes per column
    for (int c0 = 0; c0 < b;) {
        const int k = stencil_chunk(fp64, b - c0);
        const ApiOut ao{Yapi, b, c0};
        PROF_LAUNCH(h, prof_cls(kProfStencil, fp64), stencil_bytes(h->g, k, esz), st,
                    wilson_apply(h->g, fp64, Ul, kappa, (const char *)X + c0 * col,
                                 Yapi ? nullptr : (char *)Y + c0 * col, k, dagger, st, Yapi ? &ao : nullptr));
        c0 += k;
    }
    return DSBCG_OK;
}

// Y = A X on b column-major columns, T scratch of the same shape.
int apply_A_cm(dsbcg_ctx *h, bool fp64, const void *Ul, double kappa, const void *X, void *T,
               void *Y, int b, hipStream_t st) {
    CHK(stencil(h, fp64, Ul, kappa, X, T, b, false, st));
    CHK(stencil(h, fp64, Ul, kappa, T, Y, b, true, st));
    return DSBCG_OK;
}

// Structure-of-arrays copy of the caller's links.
int prepare_links(dsbcg_ctx *h, const void *U, bool fp64, hipStream_t st) {
    const int64_t V = h->g.V;
    DevBuf &buf = fp64 ? h->Ul64 : h->Ul32;
    CHK(ensure(buf, (size_t)V * 36 * (fp64 ? sizeof(zd) : sizeof(zf))));
    PROF_LAUNCH(h, kProfConvert, (double)V * 36 * (16.0 + (fp64 ? 16.0 : 8.0)), st,
                links_to_soa(V, U, buf.p, fp64, st));
    return DSBCG_OK;
}

struct SolveStats {
    int32_t block_iters = 0, rank0 = 0, deflations = 0, reliable_updates = 0, refine_iters = 0;
    int32_t final_width = 0, switch_iter = 0;
    int32_t qr2_skipped = 0;  // steps whose second CholQR pass was not needed
    int32_t qr_redone = 0;    // steps whose QR was redone column by column
    int64_t mvms = 0;
    int64_t mvms_vector = 0;      // Lanczos vectors through the stage at which the last system stopped
    std::vector<int32_t> widths;  // block width of each main-phase step
    std::vector<double> est_hist; // largest active estimate after each main-phase step
    std::vector<int32_t> frozen_at;  // [j * m + l]: Lanczos vectors through the stage at which
                                     // (l, j) stopped (0: never)
    double est[kS * kS] = {};
};

// Partial-fraction output of solve_core: Y = c0 B + sum_j c_j X_j is
// accumulated window by window and the X_j are never formed.
struct RatSpec {
    const double *coef;  // host [s]
    double c0;
    void *Yapi;          // device [V][4][3][m] FP64
};

// Initial deflated QR of the right-hand sides (M <= 256 column-major FP64
// columns in h->Bint): classical Gram-Schmidt applied twice, column by
// column, in column order.  Column l is dropped when its remainder is
// <= tau_B ||b_l|| (deflation, Sec. 1 and the deflated block Lanczos process
// of Sec. 3).  Leaves V_1 (FP64, m1 <= 16 columns) in h->V0 and rho in the
// small state; returns DSBCG_ERR_ARG with *m1_out = -1 when the rank exceeds 16.
int initial_qr(dsbcg_ctx *h, int M, double tau_B, hipStream_t st, int *m1_out) {
    const int64_t n = 12 * (int64_t)h->g.V;
    Ts ts{h, true, st, n};
    SmallState *S = stp(h);
    StepReport *rep = repp(h);
    zd *Qp = (zd *)h->Q.p;
    zd *Bp = (zd *)h->Bint.p;
    zd *wp = (zd *)h->wbuf.p;
    // ||b_l|| from the diagonals of the Gram matrices of 16-column chunks
    for (int c0 = 0; c0 < M; c0 += 16) {
        const int cnt = std::min(16, M - c0);
        TsArgs a = ts_args(n);
        a.K = 1;
        a.X[0] = Bp + (int64_t)c0 * n; a.bx[0] = cnt; a.C[0] = nullptr;
        a.bout = cnt;
        a.gram = 3;  // column norms only
        CHK(ts.run_reduce(a, cnt, 0));
        PROF_LAUNCH(h, kProfSmall, 0.0, st, small_bnorms(S, rep, red_slot(h, 0), c0, cnt, st));
    }
    int k = 0;
    for (int l = 0; l < M; ++l) {
        const zd *bl = Bp + (int64_t)l * n;
        if (k > 0) {
            // c1 = Q^H b_l
            TsArgs a = ts_args(n);
            a.K = 1;
            a.X[0] = bl; a.bx[0] = 1; a.C[0] = nullptr;
            a.bout = 1;
            a.gram = 2; a.L = Qp; a.bl = k;
            CHK(ts.run_reduce(a, k, 1));
            PROF_LAUNCH(h, kProfSmall, 0.0, st, small_neg_column(S, 0, red_slot(h, 1), k, st));
            // w = b_l - Q c1, c2 = Q^H w
            a = ts_args(n);
            a.K = 2;
            a.X[0] = bl; a.bx[0] = 1; a.C[0] = nullptr;
            a.X[1] = Qp; a.bx[1] = k; a.C[1] = coef_slot(h, 0);
            a.bout = 1;
            a.out = wp;
            a.gram = 2; a.L = Qp; a.bl = k;
            CHK(ts.run_reduce(a, k, 2));
            PROF_LAUNCH(h, kProfSmall, 0.0, st, small_neg_column(S, 1, red_slot(h, 2), k, st));
            // w = w - Q c2, ||w||^2
            a = ts_args(n);
            a.K = 2;
            a.X[0] = wp; a.bx[0] = 1; a.C[0] = nullptr;
            a.X[1] = Qp; a.bx[1] = k; a.C[1] = coef_slot(h, 1);
            a.bout = 1;
            a.out = wp;
            a.gram = 1;
            CHK(ts.run_reduce(a, 1, 3));
            PROF_LAUNCH(h, kProfSmall, 0.0, st,
                        small_cgs_decide(S, rep, red_slot(h, 1), red_slot(h, 2), red_slot(h, 3), k, l,
                                         tau_B, st));
        } else {
            TsArgs a = ts_args(n);
            a.K = 1;
            a.X[0] = bl; a.bx[0] = 1; a.C[0] = nullptr;
            a.bout = 1;
            a.out = wp;
            a.gram = 1;
            CHK(ts.run_reduce(a, 1, 3));
            PROF_LAUNCH(h, kProfSmall, 0.0, st,
                        small_cgs_decide(S, rep, nullptr, nullptr, red_slot(h, 3), 0, l, tau_B, st));
        }
        CHK(read_report(h, st));
        if (h->rep_host->flags & kFlagNonFinite)
            return fail(DSBCG_ERR_NOT_HPD, "B holds non-finite values");
        if (h->rep_host->flags & kFlagRank) {
            *m1_out = -1;
            return fail(DSBCG_ERR_ARG, "the right-hand sides span more than 16 directions");
        }
        if (h->rep_host->scalar[1] > 0.5) {
            // Q[:, k] = w / ||w||
            TsArgs a = ts_args(n);
            a.K = 1;
            a.X[0] = wp; a.bx[0] = 1; a.C[0] = coef_slot(h, 3);
            a.bout = 1;
            a.out = Qp + (int64_t)k * n;
            CHK(ts.run(a, nullptr));
            ++k;
        }
    }
    if (k > 0)
        HIPCHK(hipMemcpyAsync(h->V0.p, Qp, (size_t)n * k * sizeof(zd), hipMemcpyDeviceToDevice, st));
    *m1_out = k;
    return DSBCG_OK;
}

// Deflated QR of the b columns of W (column-major, in the data precision of
// the step) by classical Gram-Schmidt applied twice, column by column, in
// column order, into Vn: column l is kept when its remainder exceeds
// tau * ||T||_est (deflation of block vectors that became linearly
// dependent, Sec. 3).  Runs when the first CholQR pass could not resolve a
// drop decision (st->redo); leaves beta_{i+1} in R1 for small_finish and the
// kept count in *nk_out.
int redo_wqr(dsbcg_ctx *h, bool f64, const void *Wb, void *Vn, int b, double tau, hipStream_t st,
             int *nk_out) {
    const int64_t n = 12 * (int64_t)h->g.V;
    const size_t esz = f64 ? sizeof(zd) : sizeof(zf);
    Ts ts{h, f64, st, n};
    SmallState *S = stp(h);
    StepReport *rep = repp(h);
    void *wp = h->wbuf.p;  // one column of either precision
    PROF_LAUNCH(h, kProfSmall, 0.0, st, small_wqr_begin(S, st));
    WqrKept kept;
    for (int c = 0; c < kS; ++c) kept.col[c] = -1;
    int k = 0;
    for (int l = 0; l < b; ++l) {
        const void *wl = (const char *)Wb + (size_t)l * n * esz;
        if (k > 0) {
            // c1 = Q^H w
            TsArgs a = ts_args(n);
            a.K = 1;
            a.X[0] = wl; a.bx[0] = 1; a.C[0] = nullptr;
            a.bout = 1;
            a.gram = 2; a.L = Vn; a.bl = k;
            CHK(ts.run_reduce(a, k, 1));
            PROF_LAUNCH(h, kProfSmall, 0.0, st, small_neg_column(S, 0, red_slot(h, 1), k, st));
            // w' = w - Q c1, c2 = Q^H w'
            a = ts_args(n);
            a.K = 2;
            a.X[0] = wl; a.bx[0] = 1; a.C[0] = nullptr;
            a.X[1] = Vn; a.bx[1] = k; a.C[1] = coef_slot(h, 0);
            a.bout = 1;
            a.out = wp;
            a.gram = 2; a.L = Vn; a.bl = k;
            CHK(ts.run_reduce(a, k, 2));
            PROF_LAUNCH(h, kProfSmall, 0.0, st, small_neg_column(S, 1, red_slot(h, 2), k, st));
            // w'' = w' - Q c2, ||w''||^2
            a = ts_args(n);
            a.K = 2;
            a.X[0] = wp; a.bx[0] = 1; a.C[0] = nullptr;
            a.X[1] = Vn; a.bx[1] = k; a.C[1] = coef_slot(h, 1);
            a.bout = 1;
            a.out = wp;
            a.gram = 1;
            CHK(ts.run_reduce(a, 1, 3));
            PROF_LAUNCH(h, kProfSmall, 0.0, st,
                        small_wqr_decide(S, rep, red_slot(h, 1), red_slot(h, 2), red_slot(h, 3), k, l, tau, st));
        } else {
            TsArgs a = ts_args(n);
            a.K = 1;
            a.X[0] = wl; a.bx[0] = 1; a.C[0] = nullptr;
            a.bout = 1;
            a.out = wp;
            a.gram = 1;
            CHK(ts.run_reduce(a, 1, 3));
            PROF_LAUNCH(h, kProfSmall, 0.0, st,
                        small_wqr_decide(S, rep, nullptr, nullptr, red_slot(h, 3), 0, l, tau, st));
        }
        CHK(read_report(h, st));
        if (h->rep_host->scalar[1] > 0.5) {
            // Q[:, k] = w'' / ||w''||
            TsArgs a = ts_args(n);
            a.K = 1;
            a.X[0] = wp; a.bx[0] = 1; a.C[0] = coef_slot(h, 3);
            a.bout = 1;
            a.out = (char *)Vn + (size_t)k * n * esz;
            CHK(ts.run(a, nullptr));
            kept.col[k] = l;
            ++k;
        }
    }
    PROF_LAUNCH(h, kProfSmall, 0.0, st, small_wqr_end(S, rep, k, kept, st));
    *nk_out = k;
    return DSBCG_OK;
}

int check_finite_links(dsbcg_ctx *h, const void *U, hipStream_t st) {
    StepReport *rep = repp(h);
    HIPCHK(hipMemsetAsync(&rep->flags, 0, sizeof(int32_t), st));
    PROF_LAUNCH(h, kProfConvert, (double)h->g.V * 72 * 8, st,
                find_nonfinite((const double *)U, (int64_t)h->g.V * 72, &rep->flags, st));
    int32_t flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, &rep->flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (flag) return fail(DSBCG_ERR_NOT_HPD, "U holds non-finite values");
    return DSBCG_OK;
}

// Links of a call.  U != NULL: checked (optionally) and converted into the
// handle's structure-of-arrays buffers, in FP64 and, with need32, FP32; this
// replaces a copy staged by dsbcg_stage_links.  U == NULL: the staged copy
// (both precisions), which must exist.
int use_links(dsbcg_ctx *h, const void *U, bool need32, bool check, hipStream_t st) {
    if (!U) {
        if (!h->links_staged) return fail(DSBCG_ERR_ARG, "U is NULL and no links are staged on the handle");
        return DSBCG_OK;
    }
    h->links_staged = false;
    if (check) CHK(check_finite_links(h, U, st));
    CHK(prepare_links(h, U, true, st));
    if (need32) CHK(prepare_links(h, U, false, st));
    return DSBCG_OK;
}

// True relative residuals ||b_l - (sigma_j + A) x_{l,j}|| / ||b_l|| in FP64 for
// every shift (Sec. 4: relative residual); B and X in the caller's layout, the
// FP64 structure-of-arrays links in h->Ul64.  With keep_j >= 0 only that shift
// is evaluated and its residual block is stored in Rkeep (caller's layout).
// Xcm, if not NULL, holds the same iterates column-major ([s][m][n]) and is
// read instead of Xapi.
int true_residuals(dsbcg_ctx *h, hipStream_t st, double kappa, const void *Bapi, int64_t bstride,
                   const void *Xapi, int m, const double *sigma, int s, double *out, int keep_j,
                   void *Rkeep, const zd *Xcm = nullptr, const zd *Bcm = nullptr) {
    const int64_t n = 12 * (int64_t)h->g.V;
    const size_t blk = (size_t)n * m * sizeof(zd);
    CHK(ensure_common(h));
    CHK(ensure_ws(h, h->R0, blk));
    CHK(ensure_ws(h, h->R1, blk));
    CHK(ensure_ws(h, h->R2, blk));
    CHK(ensure_ws(h, h->R3, blk));
    Ts ts{h, true, st, n};
    std::vector<double> bn(m);
    std::vector<double> bn_all((size_t)s * m, 0.0);  // ||b_l|| of shift j's block
    std::vector<zd> cf(512, mk<double>(0, 0));
    // residual sums of every shift land in sums[j * 16 + l]; one copy at the end
    const int nwg = wilson_resid_workgroups(h->g);
    CHK(ensure_ws(h, h->rpart, ((size_t)nwg * 16 + 16 * (size_t)kS) * sizeof(double)));
    double *part = (double *)h->rpart.p, *sums = part + (size_t)nwg * 16;
    bool batched = false;
    const zd *bj = (const zd *)h->R0.p;  // shift j's right-hand sides, column-major
    for (int j = 0; j < s; ++j) {
        if (keep_j >= 0 && j != keep_j) continue;
        if (j == 0 || bstride != 0 || keep_j >= 0) {
            if (Bcm && keep_j < 0)
                bj = Bcm + (bstride ? (int64_t)j * n * m : 0);
            else
                CHK(copy(h, m, api((const zd *)Bapi + (int64_t)j * bstride, m), cm(h->R0.p, n, true), false, st));
            TsArgs a = ts_args(n);
            a.K = 1;
            a.X[0] = bj; a.bx[0] = m; a.C[0] = nullptr;
            a.bout = m;
            a.gram = 3;  // column norms only
            CHK(ts.run_reduce(a, m, 4));
            std::vector<zd> g(256);
            HIPCHK(hipMemcpyAsync(g.data(), red_slot(h, 4), 256 * sizeof(zd), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int l = 0; l < m; ++l) bn[l] = std::sqrt(std::max(g[l * 16 + l].x, 0.0));
        }
        const void *xj = h->R1.p;
        if (Xcm)
            xj = Xcm + (int64_t)j * n * m;
        else
            CHK(copy(h, m, api((const zd *)Xapi + (int64_t)j * n * m, m), cm(h->R1.p, n, true), false, st));
        if (keep_j < 0) {
            // D x_j, then one pass of D^H that forms |b - sigma x_j - A x_j|^2
            // per column without storing A x_j
            CHK(stencil(h, true, h->Ul64.p, kappa, xj, h->R2.p, m, false, st));
            for (int c0 = 0; c0 < m;) {
                const int k = stencil_chunk(true, m - c0);
                const int64_t off = (int64_t)c0 * n;
                PROF_LAUNCH(h, kProfStencil, stencil_bytes(h->g, k, sizeof(zd)) + (double)h->g.V * 12 * k * sizeof(zd),
                            st,
                            wilson_resid_norms(h->g, h->Ul64.p, kappa, (const zd *)h->R2.p + off, bj + off,
                                               (const zd *)xj + off, sigma[j], k,
                                               part + (size_t)c0 * nwg, st));
                c0 += k;
            }
            PROF_LAUNCH(h, kProfSmall, 0.0, st, sum_columns(part, nwg, m, sums + 16 * j, st));
            for (int l = 0; l < m; ++l) bn_all[(size_t)j * m + l] = bn[l];
            batched = true;
            continue;
        }
        CHK(apply_A_cm(h, true, h->Ul64.p, kappa, xj, h->R2.p, h->R3.p, m, st));
        TsArgs a = ts_args(n);
        a.K = 3;
        a.X[0] = h->R0.p; a.bx[0] = m; a.C[0] = nullptr;
        a.X[1] = xj; a.bx[1] = m; a.C[1] = coef_slot(h, 2);
        a.X[2] = h->R3.p; a.bx[2] = m; a.C[2] = coef_slot(h, 3);
        a.bout = m;
        a.gram = 3;  // column norms only
        if (keep_j >= 0) a.out = h->R2.p;
        // coefficient matrices -sigma_j I and -I
        for (int l = 0; l < m; ++l) {
            cf[l * 16 + l] = mk<double>(-sigma[j], 0);
            cf[256 + l * 16 + l] = mk<double>(-1.0, 0);
        }
        HIPCHK(hipMemcpyAsync((void *)coef_slot(h, 2), cf.data(), 512 * sizeof(zd),
                              hipMemcpyHostToDevice, st));
        CHK(ts.run_reduce(a, m, 5));
        if (keep_j >= 0) CHK(copy(h, m, cm(h->R2.p, n, true), api(Rkeep, m), false, st));
        std::vector<zd> g(256);
        HIPCHK(hipMemcpyAsync(g.data(), red_slot(h, 5), 256 * sizeof(zd), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int l = 0; l < m; ++l) {
            const double r = std::sqrt(std::max(g[l * 16 + l].x, 0.0));
            out[j * m + l] = bn[l] > 0 ? r / bn[l] : 0.0;
        }
    }
    if (batched) {
        std::vector<double> r2((size_t)16 * s);
        HIPCHK(hipMemcpyAsync(r2.data(), sums, (size_t)16 * s * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int j = 0; j < s; ++j)
            for (int l = 0; l < m; ++l) {
                const double b = bn_all[(size_t)j * m + l];
                out[j * m + l] = b > 0 ? std::sqrt(std::max(r2[(size_t)16 * j + l], 0.0)) / b : 0.0;
            }
    }
    return DSBCG_OK;
}

// The DSBlockCG iteration.  FP64 form: every vector in FP64.  FP32 form: the
// iteration starts in FP64 and continues the same recurrences with FP32
// vectors once every active estimate is <= switch_at.  The iterates are
// formed window by window from the kept Lanczos blocks (FP32 blocks
// contracted in FP32) and accumulated in FP64; a window of FP32 blocks ends
// at least every ru_interval steps.  Writes the iterates to Xapi
// ([s][V][4][3][m], FP64), or with rat their partial-fraction sum to
// rat->Yapi.  The FP64 links must be in h->Ul64 (and the FP32 links in
// h->Ul32 for the FP32 form).
int solve_core(dsbcg_ctx *h, double kappa, const void *B, int64_t bstride, int m,
               const double *sigma, int s, double tol, const dsbcg_opts &o, double switch_at,
               void *Xapi, SolveStats &stt, hipStream_t st, const RatSpec *rat) {
    const int64_t V = h->g.V, n = 12 * V;
    const bool form32 = o.precision == DSBCG_FP32_RELIABLE;
    // drop threshold of steps run with FP32 vectors: an exactly dependent
    // direction keeps a remainder of a few FP32 units of ||w|| after
    // orthogonalisation, which 1e-5 ||T||_est clears with a wide margin
    const double tau32 = std::max(o.tau_W, kTauW32);
    const int M = bstride ? m * s : m;  // stacked right-hand-side columns
    const bool rmode = rat != nullptr;  // partial-fraction output, no X_j
    if (rmode && (form32 || bstride != 0))
        return fail(DSBCG_ERR_ARG, "internal: the partial-fraction form runs in FP64 on one B");

    CHK(ensure_common(h));
    CHK(ensure_ws(h, h->Bint, (size_t)n * M * sizeof(zd)));
    CHK(ensure_ws(h, h->Q, (size_t)n * std::min(M, (int)kS) * sizeof(zd)));
    CHK(ensure_ws(h, h->wbuf, (size_t)n * sizeof(zd)));
    CHK(ensure_ws(h, h->V0, (size_t)n * std::min(M, (int)kS) * sizeof(zd)));
    if (!rmode) CHK(ensure_ws(h, h->X, (size_t)n * m * s * sizeof(zd)));

    SmallState *S = stp(h);
    StepReport *rep = repp(h);
    HIPCHK(hipMemsetAsync(rep, 0, sizeof(StepReport), st));
    for (int j = 0; j < (bstride ? s : 1); ++j)
        CHK(copy(h, m, api((const zd *)B + (int64_t)j * bstride, m),
                 cm((zd *)h->Bint.p + (int64_t)j * m * n, n, true), false, st));
    if (rmode) {
        // Y = c0 B; the windows add sum_j c_j X_j
        CHK(ensure_ws(h, h->Ycm, (size_t)n * m * sizeof(zd)));
        CHK(ensure(h->ycoef, kS * sizeof(double)));
        std::vector<double> cf(kS, 0.0);
        for (int j = 0; j < s; ++j) cf[j] = rat->coef[j];
        HIPCHK(hipMemcpyAsync(h->ycoef.p, cf.data(), kS * sizeof(double), hipMemcpyHostToDevice, st));
        PROF_LAUNCH(h, kProfConvert, copy_bytes(V, m, 16, 16, false), st,
                    copy_field(V, m, cm(h->Bint.p, n, true), cm(h->Ycm.p, n, true), false, rat->c0, st));
    }

    int m1 = 0;
    CHK(initial_qr(h, M, o.tau_B, st, &m1));
    stt.rank0 = m1;
    PROF_LAUNCH(h, kProfSmall, 0.0, st,
                small_init_shifts(S, rep, m1, m, s, sigma, o.freeze, tol, bstride != 0, st));
    CHK(read_report(h, st));

    // widths never exceed m1 after the initial deflation
    const int wmax = std::max(m1, 1);
    const int steps = o.fixed_iters > 0 ? o.fixed_iters : o.max_iters;
    const size_t b64 = (size_t)n * wmax * sizeof(zd), b32 = (size_t)n * wmax * sizeof(zf);
    CHK(ensure_ws(h, h->T, b64));
    CHK(ensure_ws(h, h->W, b64));
    if (form32) {
        CHK(ensure_ws(h, h->T32, b32));
        CHK(ensure_ws(h, h->W32, b32));
    }
    // the P_j buffers (s blocks of the widest width, two per precision) are
    // allocated when a window first forms or reads them: a solve that one
    // window covers never does
    // (plain ensure: the window rings hold live blocks by then and must not
    // be released to make room)
    auto ensure_p = [&](bool f64s) -> int {
        if (f64s) {
            CHK(ensure(h->P[0], b64 * s));
            CHK(ensure(h->P[1], b64 * s));
        } else {
            CHK(ensure(h->P32[0], b32 * s));
            CHK(ensure(h->P32[1], b32 * s));
        }
        return DSBCG_OK;
    };
    CHK(ensure(h->wcoef, wincoef_bytes()));
    CHK(ensure(h->wlist, 64 * sizeof(int32_t)));
    const WinCoef WC = wincoef_at(h->wcoef.p);

    // Window length K: the Lanczos blocks of up to K steps are kept and the
    // per-shift iterates are formed from them once per window.  Three
    // quarters of the free device memory (counting the rings this handle
    // already holds), less 4 GiB, is the budget; the FP32 phase also flushes
    // into the FP64 solution at least every ru_interval steps.
    int K64 = 1, K32 = 1;
    {
        size_t freeb = 0, totalb = 0;
        HIPCHK(hipMemGetInfo(&freeb, &totalb));
        double held = 0.0;
        for (const DevBuf &r : h->Vring) held += (double)r.bytes;
        for (const DevBuf &r : h->Vring32) held += (double)r.bytes;
        const double budget = 0.75 * ((double)freeb + held) - 4.0 * (1 << 30);
        const double per_step = (double)b64 + (form32 ? (double)b32 : 0.0);
        const double kfit = std::floor(budget / per_step) - 2.0;
        int K = (int)std::min<double>((double)kWinMax, kfit);
        if (o.window > 0) K = std::min(K, o.window);
        K = std::min(K, steps);
        if (K < 1) return fail(DSBCG_ERR_OOM, "not enough device memory for the Lanczos blocks of a window");
        K64 = K;
        K32 = std::min(K, std::max(1, o.ru_interval));
    }
    const int nring64 = K64 + 2, nring32 = form32 ? K32 + 2 : 0;
    // the budget counted every block the rings hold: give back the ones this
    // solve does not use before allocating the others
    for (size_t k = nring64; k < h->Vring.size(); ++k)
        if (h->Vring[k].p) {
            HIPCHK(hipFree(h->Vring[k].p));
            h->Vring[k].p = nullptr;
            h->Vring[k].bytes = 0;
        }
    for (size_t k = nring32; k < h->Vring32.size(); ++k)
        if (h->Vring32[k].p) {
            HIPCHK(hipFree(h->Vring32[k].p));
            h->Vring32[k].p = nullptr;
            h->Vring32[k].bytes = 0;
        }
    if ((int)h->Vring.size() < nring64) h->Vring.resize(nring64);
    if ((int)h->Vring32.size() < nring32) h->Vring32.resize(nring32);
    // slots are allocated when a step first takes them (slot_in), so a solve
    // holds only the blocks its windows keep
    std::vector<void *> ring64(nring64, nullptr), ring32(nring32, nullptr);
    ring64[0] = h->V0.p;
    auto slot_in = [&](bool f64s, int k) -> int {
        if (f64s) {
            if (!ring64[k]) {
                CHK(ensure(h->Vring[k], b64));
                ring64[k] = h->Vring[k].p;
            }
        } else if (!ring32[k]) {
            CHK(ensure(h->Vring32[k], b32));
            ring32[k] = h->Vring32[k].p;
        }
        return DSBCG_OK;
    };
    // coefficient tables and window column pointers, sized for the longest
    // window (FP64 part and FP32 part each get their own region)
    const int kwin = std::min((int)kWinMax, K64 + (form32 ? K32 : 0));
    const int npairs_max = (wmax + 1) / 2 + (kwin * wmax + 1) / 2 + 1;
    CHK(ensure(h->wtable, (size_t)2 * s * npairs_max * 4 * 64 * sizeof(double)));
    CHK(ensure(h->colptr, (size_t)(kwin * wmax + 2) * sizeof(void *)));
    bool lo = false;
    PROF_LAUNCH(h, kProfSmall, 0.0, st, small_window_reset(WC, st));

    // Lanczos blocks by step: v64[i] / v32[i] = slot of V_i in the FP64 / FP32
    // ring (-1: none), bw[i] = width.  After the switch to FP32 vectors the
    // window's FP64 blocks stay in their ring until the window ends.
    std::vector<int> v64(2, -1), v32(2, -1), bw(2, 0);
    std::vector<int> free64, free32;
    for (int k = nring64 - 1; k >= 1; --k) free64.push_back(k);
    v64[1] = 0;
    bw[1] = m1;
    auto ring = [&](int i) -> void * { return lo ? ring32[v32[i]] : ring64[v64[i]]; };
    int sw = 0;  // first step of the current window run with FP32 vectors (0: none)

    int b = m1, bp = 0;
    int pcur = 0;        // P buffer holding P_{j,i0}
    int i0 = 0;          // the current window covers steps i0+1 .. i
    std::vector<int32_t> wset;  // shifts updated in the current window
    int status = DSBCG_OK;
    int iters = 0;
    std::vector<int32_t> act;
    std::vector<void *> colptr_host;
    // vector-wise stopping: small_finish leaves the masks alone and
    // small_vector_stop stops each system at its own Lanczos vector
    const bool vstop = o.freeze && o.vector_stop;
    const int finish_freeze = vstop ? 0 : o.freeze;
    int64_t kvec = 0;  // Lanczos vectors before the current block
    stt.frozen_at.assign((size_t)s * m, 0);
    std::vector<uint32_t> mask_in(s, 0), mask0(s);
    for (int j = 0; j < s; ++j) mask_in[j] = h->rep_host->colmask[j];
    bool xfresh = true;  // X has not been written yet in this solve
    // shifts whose X_j the last window already stored in the caller's layout
    std::vector<char> api_done(s, 0);

    auto active_list = [&](void) {
        act.clear();
        for (int j = 0; j < s; ++j)
            if (h->rep_host->colmask[j]) act.push_back(j);
    };
    auto max_active_est = [&](void) {
        double e = 0.0;
        for (int j : act)
            for (int l = 0; l < m; ++l)
                if ((h->rep_host->colmask[j] >> l) & 1u) e = std::max(e, h->rep_host->est[j][l]);
        return e;
    };
    auto release = [&](int i) {
        // V_{i0} .. V_{i-1} are no longer needed once the window ends at step i
        for (int k = std::max(i0, 1); k < i; ++k) {
            if (v64[k] >= 0) {
                free64.push_back(v64[k]);
                v64[k] = -1;
            }
            if (v32[k] >= 0) {
                free32.push_back(v32[k]);
                v32[k] = -1;
            }
        }
        i0 = i;
        sw = 0;
    };
    // Apply the window i0+1 .. i to X_j, and form P_{j,i} for the shifts
    // still active when the iteration goes on (need_p).  A window that spans
    // the switch to FP32 vectors runs as two contractions: blocks up to sw in
    // FP64 (with the P_{j,i0} term), the later ones in FP32; their P parts
    // are added in FP32.
    auto apply_window = [&](int i, bool need_p) -> int {
        if (wset.empty() || i <= i0) {
            release(i);
            wset = act;
            return DSBCG_OK;
        }
        if (need_p || i0 >= 1) {
            // P_{j,i0} is read or P_{j,end} formed
            CHK(ensure_p(true));
            if (lo || sw > 0) CHK(ensure_p(false));
        }
        // the last window of the solve also writes its shifts' X_j to the caller
        zd *xapi = (!need_p && !rmode && Xapi) ? (zd *)Xapi : nullptr;
        std::vector<int32_t> pm(s, 0);
        if (need_p)
            for (int j : act) pm[j] = 1;
        const int bend = (need_p && !act.empty()) ? bw[i] : 0;
        int32_t *wl = h->list_host + 64;  // pinned: window shift list, then P flags
        for (size_t q = 0; q < wset.size(); ++q) wl[q] = wset[q];
        for (int j = 0; j < s; ++j) wl[16 + j] = pm[j];
        HIPCHK(hipMemcpyAsync(h->wlist.p, wl, 64 * sizeof(int32_t), hipMemcpyHostToDevice, st));
        const int32_t *dshift = (const int32_t *)h->wlist.p, *dpm = dshift + 16;
        if (xfresh && !rmode) {
            // the first window writes X_j of its shifts; the others start from zero
            std::vector<char> in_w(s, 0);
            for (int j : wset) in_w[j] = 1;
            for (int j = 0; j < s; ++j)
                if (!in_w[j])
                    HIPCHK(hipMemsetAsync((zd *)h->X.p + (int64_t)j * n * m, 0, (size_t)n * m * sizeof(zd), st));
        }
        // segments: [first step, last step, precision]
        struct Seg { int a, b; bool f64; };
        std::vector<Seg> seg;
        if (sw > 0) {
            seg.push_back({i0 + 1, std::min(sw, i), true});
            if (i > sw) seg.push_back({sw + 1, i, false});
        } else {
            seg.push_back({i0 + 1, i, !lo});
        }
        // both segments' pointers are copied from one host array: reserve it
        // so the first copy's source is not moved by the second segment
        colptr_host.clear();
        colptr_host.reserve((size_t)(i - i0) * wmax);
        size_t tab_off = 0;  // elements (doubles) into the table buffer
        WinArgs wfirst;      // FP64 part of a window across the switch
        memset(&wfirst, 0, sizeof(wfirst));
        // three real products per complex product where the window has no
        // P_{j,i0} inputs and at most 8 outputs per shift (both parts of a
        // window across the switch take the same form)
        const bool gauss = !rmode && (i0 < 1 || bw[i0] == 0) && m + bend <= 8;
        double bytes_first = 0.0;
        const int pnew = pcur ^ 1;
        for (size_t sg = 0; sg < seg.size(); ++sg) {
            const Seg &g = seg[sg];
            const bool f64s = g.f64;
            const size_t esz = f64s ? sizeof(zd) : sizeof(zf);
            WindowTable wt;
            memset(&wt, 0, sizeof(wt));
            wt.nshift = (int)wset.size();
            wt.bp0 = (sg == 0 && i0 >= 1) ? bw[i0] : 0;
            wt.m = m;
            wt.K = g.b - g.a + 1;
            wt.slot0 = g.a - i0 - 1;
            const size_t cp0 = colptr_host.size();
            for (int u = 0; u < wt.K; ++u) {
                const int step = g.a + u;
                const int w = bw[step];
                wt.wb[u] = w;
                void *base = f64s ? ring64[v64[step]] : ring32[v32[step]];
                for (int c = 0; c < w; ++c) colptr_host.push_back((char *)base + (size_t)c * n * esz);
            }
            wt.ncolv = (int)(colptr_host.size() - cp0);
            wt.bend = bend;
            wt.pairs_p = (wt.bp0 + 1) / 2;
            wt.npairs = wt.pairs_p + (wt.ncolv + 1) / 2;
            wt.nmt = (m + wt.bend + 7) / 8;
            void **dcol = (void **)h->colptr.p + cp0;
            if (wt.ncolv > 0)
                HIPCHK(hipMemcpyAsync(dcol, colptr_host.data() + cp0, (size_t)wt.ncolv * sizeof(void *),
                                      hipMemcpyHostToDevice, st));
            if (rmode) {
                // P_{j,end} of the shifts going on, then Y += sum_j c_j (increment of X_j)
                if (bend > 0) {
                    WindowTable wp = wt;
                    wp.m = 0;
                    wp.nmt = (bend + 7) / 8;
                    double *tab = (double *)h->wtable.p + tab_off;
                    tab_off += (size_t)wp.nshift * wp.npairs * wp.nmt * 64;
                    PROF_LAUNCH(h, kProfSmall, 0.0, st, small_window_table(WC, wp, dshift, dpm, true, tab, st));
                    WinArgs wa;
                    memset(&wa, 0, sizeof(wa));
                    wa.nrows = n;
                    wa.ncolv = wp.ncolv;
                    wa.colptr = (const void *const *)dcol;
                    wa.bp0 = wp.bp0;
                    wa.Pold = h->P[pcur].p;
                    wa.Pnew = h->P[pnew].p;
                    wa.bend = bend;
                    wa.pstride = n * wmax;
                    wa.m = 0;
                    wa.X = (zd *)h->Ycm.p;  // not written with m = 0
                    wa.xstride = 0;
                    wa.table = tab;
                    wa.npairs = wp.npairs;
                    wa.pairs_p = wp.pairs_p;
                    wa.nmt = wp.nmt;
                    wa.shifts = dshift;
                    wa.nshift = wp.nshift;
                    wa.xmask = WC.Wmask;
                    wa.pmask = dpm;
                    const double bytes =
                        (double)n * sizeof(zd) * (wp.ncolv + wp.nshift * (wp.bp0 + bend));
                    PROF_LAUNCH(h, kProfShift, bytes, st, window_apply(true, wa, st));
                }
                RatArgs ra;
                memset(&ra, 0, sizeof(ra));
                ra.nrows = n;
                ra.ncolv = wt.ncolv;
                ra.colptr = (const void *const *)dcol;
                ra.bp0 = wt.bp0;
                ra.Pold = h->P[pcur].p;
                ra.pstride = n * wmax;
                ra.shifts = dshift;
                ra.nshift = wt.nshift;
                ra.m = m;
                ra.Y = (zd *)h->Ycm.p;
                ra.pairs_p = wt.pairs_p;
                ra.npairs = wt.nshift * wt.pairs_p + (wt.ncolv + 1) / 2;
                ra.nmt = (m + 7) / 8;
                double *tab = (double *)h->wtable.p + tab_off;
                tab_off += (size_t)ra.npairs * ra.nmt * 64;
                ra.table = tab;
                PROF_LAUNCH(h, kProfSmall, 0.0, st,
                            small_rational_table(WC, wt, dshift, (const double *)h->ycoef.p, true, tab, st));
                const double bytes = (double)n * sizeof(zd) * (wt.ncolv + wt.nshift * wt.bp0 + 2.0 * m);
                PROF_LAUNCH(h, kProfShift, bytes, st, rational_window_apply(true, ra, st));
                continue;
            }
            double *tab = (double *)h->wtable.p + tab_off;
            // the FP32 part of a window across the switch keeps the real
            // 2 x 2 table (see WinArgs.gauss)
            if (gauss && !(seg.size() == 2 && sg == 1)) {
                tab_off += (size_t)((wt.nshift + 1) / 2) * ((wt.ncolv + 3) / 4) * 3 * 64;
                PROF_LAUNCH(h, kProfSmall, 0.0, st, small_window_table3(WC, wt, dshift, dpm, f64s, tab, st));
            } else {
                tab_off += (size_t)wt.nshift * wt.npairs * wt.nmt * 64;
                PROF_LAUNCH(h, kProfSmall, 0.0, st, small_window_table(WC, wt, dshift, dpm, f64s, tab, st));
            }
            WinArgs wa;
            memset(&wa, 0, sizeof(wa));
            wa.nrows = n;
            wa.ncolv = wt.ncolv;
            wa.colptr = (const void *const *)dcol;
            wa.bp0 = wt.bp0;
            // P_{j,i0} is in the precision the window started in
            wa.Pold = f64s ? h->P[pcur].p : h->P32[pcur].p;
            wa.Pnew = f64s ? h->P[pnew].p : h->P32[pnew].p;
            wa.bend = wt.bend;
            wa.pstride = n * wmax;
            wa.m = m;
            wa.X = (zd *)h->X.p;
            wa.xstride = n * m;
            wa.table = tab;
            wa.npairs = wt.npairs;
            wa.pairs_p = wt.pairs_p;
            wa.nmt = wt.nmt;
            wa.shifts = dshift;
            wa.nshift = wt.nshift;
            wa.xmask = WC.Wmask;
            wa.pmask = dpm;
            wa.xinit = (xfresh && sg == 0) ? 1 : 0;
            wa.Xapi = xapi;
            wa.gauss = gauss ? 1 : 0;
            const double api_bytes = xapi ? (double)n * sizeof(zd) * m * wt.nshift : 0.0;
            if (seg.size() == 2 && sg == 0) {
                // a window across the switch: the FP64 part waits for the FP32
                // part and both run as one launch that writes X_j once
                wfirst = wa;
                bytes_first = (double)n * esz * (wt.ncolv + wt.nshift * wt.bp0);
                continue;
            }
            if (seg.size() == 2) {
                WinArgs w2 = wfirst;
                w2.ncolv2 = wa.ncolv;
                w2.colptr2 = wa.colptr;
                w2.table2 = wa.table;
                w2.npairs2 = wa.npairs;
                w2.Pnew2 = h->P32[pnew].p;
                // the iteration goes on in FP32: P_{j,end} (both parts) is written in FP32
                const double bytes = bytes_first + api_bytes +
                                     (double)n * ((double)esz * (wt.ncolv + wt.nshift * wt.bend) +
                                                  (w2.xinit ? 1.0 : 2.0) * sizeof(zd) * m * wt.nshift);
                PROF_LAUNCH(h, prof_cls(kProfShift, true), bytes, st, window_apply(true, w2, st));
                stt.reliable_updates += 1;
                continue;
            }
            const double bytes = api_bytes +
                                 (double)n * ((double)esz * (wt.ncolv + wt.nshift * (wt.bp0 + wt.bend)) +
                                              (wa.xinit ? 1.0 : 2.0) * sizeof(zd) * m * wt.nshift);
            PROF_LAUNCH(h, prof_cls(kProfShift, f64s), bytes, st, window_apply(f64s, wa, st));
            if (!f64s) stt.reliable_updates += 1;
        }
        xfresh = false;
        if (xapi)
            for (int j : wset) api_done[j] = 1;
        if (sw > 0 && bend > 0 && seg.size() == 1)
            // the window ended at the switch step: P_{j,i} leaves the FP64 part in FP32
            for (int j : act)
                CHK(copy(h, bend, cm((zd *)h->P[pnew].p + (int64_t)j * n * wmax, n, true),
                         cm((zf *)h->P32[pnew].p + (int64_t)j * n * wmax, n, false), false, st));
        // the host buffers are rewritten only after the next step's report,
        // which waits for the stream
        pcur = pnew;
        release(i);
        wset = act;
        return DSBCG_OK;
    };
    active_list();
    wset = act;
    bool done = (m1 == 0) || (act.empty() && o.fixed_iters <= 0);

    for (int i = 1; !done && i <= steps; ++i) {
        if (form32 && !lo && max_active_est() <= switch_at) {
            // continue the same recurrences with FP32 vectors: V_{i-1} and V_i
            // get FP32 copies.  An open window keeps its FP64 blocks and goes
            // on (its P_{j,i0} stays FP64); a window that ended with the
            // previous step hands over P_{j,i-1} in FP32.
            free32.clear();
            for (int k = nring32 - 1; k >= 2; --k) free32.push_back(k);
            CHK(slot_in(false, 1));
            CHK(copy(h, b, cm(ring64[v64[i]], n, true), cm(ring32[1], n, false), false, st));
            v32[i] = 1;
            {
                // the Gram of V_i as rounded to FP32 (slot 3) for the next Gram correction
                Ts ts32{h, false, st, n};
                TsArgs a = ts_args(n);
                a.K = 1;
                a.X[0] = ring32[1]; a.bx[0] = b; a.C[0] = nullptr;
                a.bout = b;
                a.gram = 1;
                CHK(ts32.run_reduce(a, b, 3));
                PROF_LAUNCH(h, kProfSmall, 0.0, st, small_set_nv(S, red_slot(h, 3), st));
            }
            if (i > 1) {
                CHK(slot_in(false, 0));
                CHK(copy(h, bp, cm(ring64[v64[i - 1]], n, true), cm(ring32[0], n, false), false, st));
                v32[i - 1] = 0;
            } else {
                free32.push_back(0);
            }
            if (i0 < i - 1) {
                sw = i;
            } else if (i > 1) {
                CHK(ensure_p(false));
                for (int j : act)
                    CHK(copy(h, bp, cm((zd *)h->P[pcur].p + (int64_t)j * n * wmax, n, true),
                             cm((zf *)h->P32[pcur].p + (int64_t)j * n * wmax, n, false), false, st));
            }
            lo = true;
            stt.switch_iter = i;
        }
        const bool f64 = !lo;
        Ts ts{h, f64, st, n};
        for (int j = 0; j < s; ++j) mask0[j] = h->rep_host->colmask[j];
        iters = i;
        stt.mvms += b;
        stt.widths.push_back(b);
        if ((int)v64.size() < i + 2) {
            v64.resize(i + 2, -1);
            v32.resize(i + 2, -1);
            bw.resize(i + 2, 0);
        }
        std::vector<int> &fl = lo ? free32 : free64;
        if (fl.empty()) {
            status = fail(DSBCG_ERR_HIP, "internal: Lanczos block ring exhausted");
            break;
        }
        (lo ? v32 : v64)[i + 1] = fl.back();
        CHK(slot_in(!lo, fl.back()));
        fl.pop_back();
        void *Vc = ring(i), *Vp = i > 1 ? ring(i - 1) : ring(i), *Vn = ring(i + 1);
        void *T = lo ? h->T32.p : h->T.p, *Wb = lo ? h->W32.p : h->W.p;
        const void *Ul = lo ? h->Ul32.p : h->Ul64.p;
    // W = A V_i
        CHK(apply_A_cm(h, f64, Ul, kappa, Vc, T, Wb, b, st));
        // One pass over W, V_{i-1}, V_i: W' = W - V_{i-1} beta_i^H (not stored),
        // M = V_i^H W' (slot 0) and G' = W'^H W' (slot 1).
        const double col_bytes = (double)n * (f64 ? sizeof(zd) : sizeof(zf));
        {
            TsArgs a = ts_args(n);
            a.K = (i > 1) ? 2 : 1;
            a.X[0] = Wb; a.bx[0] = b; a.C[0] = nullptr;
            a.X[1] = Vp; a.bx[1] = bp; a.C[1] = coef_slot(h, 0);
            a.bout = b;
            a.gram = 4; a.L = Vc; a.bl = b;
            CHK(ts.run_reduce(a, b, 0));
        }
        // alpha_i = herm(M), -alpha_i as a coefficient; the Gram of
        // W'' = W' - V_i alpha_i from M, G' and alpha_i (slot 2)
        PROF_LAUNCH(h, kProfSmall, 0.0, st, small_prep_alpha(S, red_slot(h, 0), st));
        PROF_LAUNCH(h, kProfSmall, 0.0, st, small_lanczos_gram(S, red_slot(h, 0), red_slot(h, 1), red_slot(h, 2), st));
        // per-shift coefficients and the window recurrences
        for (size_t q = 0; q < act.size(); ++q) h->list_host[q] = act[q];
        HIPCHK(hipMemcpyAsync(h->list.p, h->list_host, act.size() * sizeof(int32_t) + 4,
                              hipMemcpyHostToDevice, st));
        PROF_LAUNCH(h, kProfSmall, 0.0, st,
                    small_shift_coeffs(S, rep, red_slot(h, 0), i == 1, (const int32_t *)h->list.p,
                                       (int)act.size(), st));
        WindowStep wsp;
        {
            wsp.t = i - i0 - 1;
            wsp.bp0 = i0 >= 1 ? bw[i0] : 0;
            wsp.b = b;
            wsp.bp = bp;
            wsp.m = m;
            bw[i] = b;
            PROF_LAUNCH(h, kProfSmall, 0.0, st,
                        small_window_update(S, rep, WC, wsp, (const int32_t *)h->list.p, (int)act.size(), st));
        }
        // vector-wise stopping after small_finish: the stage estimates inside
        // this block, and the window coefficients of the systems that stop
        // before its last vector
        auto vector_stop = [&](void) -> int {
            if (!vstop) return DSBCG_OK;
            PROF_LAUNCH(h, kProfSmall, 0.0, st,
                        small_vector_stop(S, rep, tol, (const int32_t *)h->list.p, (int)act.size(), st));
            PROF_LAUNCH(h, kProfSmall, 0.0, st,
                        small_window_correct(S, WC, wsp, (const int32_t *)h->list.p, (int)act.size(), st));
            return DSBCG_OK;
        };
        // first CholQR pass with deflation on the Gram of W''
        PROF_LAUNCH(h, kProfSmall, 0.0, st,
                    small_chol_deflate(S, rep, red_slot(h, 0), red_slot(h, 2), lo ? tau32 : o.tau_W, st,
                                       red_slot(h, 1)));
        PROF_LAUNCH(h, kProfSmall, 0.0, st, small_basis_coefs(S, st));
        // V' = W'' C1 = W C1 - V_i alpha_i C1 - V_{i-1} beta_i^H C1 into V_{i+1}'s
        // slot, with its Gram G2 = V'^H V' (slot 3) from the values stored:
        // the first bnew columns are the new block (the others are zero and
        // never read).  Skipped on the device when the step's QR has to be
        // redone column by column.
        {
            TsArgs a = ts_args(n);
            a.K = (i > 1) ? 3 : 2;
            a.X[0] = Wb; a.bx[0] = b; a.C[0] = S->cB[0];
            a.X[1] = Vc; a.bx[1] = b; a.C[1] = S->cB[1];
            a.X[2] = Vp; a.bx[2] = bp; a.C[2] = S->cB[2];
            a.bout = b;
            a.out = Vn;
            a.gram = 1;
            a.skip = &S->redo;
            CHK(ts.run_reduce(a, b, 3));
        }
        // second CholQR pass, only when the kept columns are ill-conditioned
        // (skipped on the device otherwise): V_{i+1} = V' R2^{-1}, R2 from G2
        PROF_LAUNCH(h, kProfSmall, 0.0, st,
                    small_finish(S, rep, red_slot(h, 3), tol, finish_freeze, (const int32_t *)h->list.p,
                                 (int)act.size(), st));
        CHK(vector_stop());
        {
            TsArgs a = ts_args(n);
            a.K = 1;
            a.X[0] = Vn; a.bx[0] = b; a.C[0] = S->R2inv;
            a.bout = b;
            a.out = Vn;  // in place: every thread reads its rows before writing them
            a.skip = &S->skip_qr2;
            CHK(ts.run(a, nullptr));
        }
        CHK(read_report(h, st));
        if (prof_on(h, prof_cls(kProfBlock, f64)) && h->rep_host->skip_qr2) {
            // the second-pass launch returned at once: it moved no data
            const int cls = prof_cls(kProfBlock, f64);
            h->prof_bytes[cls] -= 2.0 * b * col_bytes;
            h->prof_launches[cls] -= 1;
        }
        if (h->rep_host->flags & kFlagRedoQR) {
            // a drop decision below the resolution of the Gram matrix: the
            // skipped basis update moved no data; form W'' and redo its QR
            // column by column
            if (prof_on(h, prof_cls(kProfBlock, f64))) {
                const int cls = prof_cls(kProfBlock, f64);
                h->prof_bytes[cls] -= (3.0 * b + bp) * col_bytes;
                h->prof_launches[cls] -= 1;
            }
            {
                TsArgs a = ts_args(n);
                a.K = (i > 1) ? 3 : 2;
                a.X[0] = Wb; a.bx[0] = b; a.C[0] = nullptr;
                a.X[1] = Vc; a.bx[1] = b; a.C[1] = coef_slot(h, 1);
                a.X[2] = Vp; a.bx[2] = bp; a.C[2] = coef_slot(h, 0);
                a.bout = b;
                a.out = Wb;
                CHK(ts.run(a, nullptr));
            }
            int nk = 0;
            CHK(redo_wqr(h, f64, Wb, Vn, b, lo ? tau32 : o.tau_W, st, &nk));
            if (nk > 0) {
                // Gram of the new block as stored (slot 3), kept for the next step
                TsArgs a = ts_args(n);
                a.K = 1;
                a.X[0] = Vn; a.bx[0] = nk; a.C[0] = nullptr;
                a.bout = nk;
                a.gram = 1;
                CHK(ts.run_reduce(a, nk, 3));
            }
            PROF_LAUNCH(h, kProfSmall, 0.0, st,
                        small_finish(S, rep, red_slot(h, 3), tol, finish_freeze, (const int32_t *)h->list.p,
                                     (int)act.size(), st));
            CHK(vector_stop());
            CHK(read_report(h, st));
            stt.qr_redone += 1;
        }
        const StepReport &R = *h->rep_host;
        stt.qr2_skipped += R.skip_qr2 ? 1 : 0;
        if (R.flags & kFlagNotHPD) {
            status = fail(DSBCG_ERR_NOT_HPD, "shifted block lost positive definiteness at step " +
                                                 std::to_string(i) + ": sigma_j I + A is not hpd");
            break;
        }
        if (R.flags & kFlagQR2) {
            status = fail(DSBCG_ERR_NOT_CONVERGED,
                          "orthonormalisation of the Lanczos block failed at step " + std::to_string(i));
            break;
        }
        const int bnew = R.bnew;
        stt.deflations += b - bnew;
        for (int j = 0; j < s; ++j)
            for (int l = 0; l < m; ++l)
                if (((mask0[j] >> l) & 1u) && !((R.colmask[j] >> l) & 1u))
                    stt.frozen_at[(size_t)j * m + l] = (int32_t)(kvec + (vstop ? R.stage[j][l] : b));
        kvec += b;
        {
            // residual history: the worst estimate among the systems that
            // were updated in this step
            double e = 0.0;
            for (int j = 0; j < s; ++j)
                for (int l = 0; l < m; ++l)
                    if ((mask0[j] >> l) & 1u) e = std::max(e, R.est[j][l]);
            stt.est_hist.push_back(e);
        }
        active_list();
        if (bnew == 0) done = true;
        if (o.fixed_iters <= 0 && act.empty()) done = true;
        // the window ends when a ring is full, at the slot limit, or at the end
        const bool full = lo ? (i - std::max(i0, sw > 0 ? sw - 1 : i0) >= K32) : (i - i0 >= K64);
        if (full || i - i0 >= kwin || done || i == steps) CHK(apply_window(i, !done && i < steps));
        bp = b;
        b = bnew;
        bw[i + 1] = bnew;
        stt.final_width = bnew;
    }
    if (xfresh && !rmode)  // no window was applied (no step, or nothing to update)
        HIPCHK(hipMemsetAsync(h->X.p, 0, (size_t)n * m * s * sizeof(zd), st));
    stt.block_iters += iters;
    {
        // the stage at which the last system stopped (all of them did), else
        // every Lanczos vector of the run
        bool all = true;
        int64_t last = 0;
        for (int j = 0; j < s; ++j)
            for (int l = 0; l < m; ++l)
                if ((mask_in[j] >> l) & 1u) {
                    const int32_t f = stt.frozen_at[(size_t)j * m + l];
                    all = all && f > 0;
                    last = std::max<int64_t>(last, f);
                }
        stt.mvms_vector = all ? last : kvec;
    }
    if (status == DSBCG_OK && !done && o.fixed_iters <= 0)
        status = fail(DSBCG_ERR_NOT_CONVERGED, "max_iters reached");
    // iterates (or their partial-fraction sum) to the caller's layout
    if (rmode)
        CHK(copy(h, m, cm(h->Ycm.p, n, true), api(rat->Yapi, m), false, st));
    else
        for (int j = 0; j < s; ++j)
            if (!api_done[j])
                CHK(copy(h, m, cm((zd *)h->X.p + (int64_t)j * n * m, n, true),
                         api((zd *)Xapi + (int64_t)j * n * m, m), false, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int j = 0; j < s; ++j)
        for (int l = 0; l < m; ++l) stt.est[j * m + l] = h->rep_host->est[j][l];
    return status;
}

int check_field_args(dsbcg_handle h, const void *U, const void *X, const void *Y, int32_t m,
                     double kappa) {
    if (!h || !X || !Y) return fail(DSBCG_ERR_ARG, "NULL argument");
    if (!U && !h->links_staged) return fail(DSBCG_ERR_ARG, "U is NULL and no links are staged on the handle");
    if (m < 1 || m > DSBCG_MAX_RHS) return fail(DSBCG_ERR_ARG, "m out of range");
    if (!std::isfinite(kappa)) return fail(DSBCG_ERR_ARG, "kappa not finite");
    if (X == Y) return fail(DSBCG_ERR_ARG, "Y must not alias X");
    return DSBCG_OK;
}

}  // namespace

extern "C" {

void dsbcg_default_opts(dsbcg_opts *o) {
    if (!o) return;
    o->precision = DSBCG_FP64;
    o->max_iters = 10000;
    o->fixed_iters = 0;
    o->ru_interval = 50;
    o->tau_B = -1.0;      // resolved to 0.1 * tol
    o->tau_W = -1.0;      // resolved to 1e-12
    o->refine = 1;
    o->freeze = 1;
    o->switch_at = -1.0;  // resolved to min(1e-2, 1e5 * tol)
    o->window = 0;        // automatic window length
    o->keep_workspace = 1;
    o->vector_stop = 0;   // stop systems at block boundaries
}

const char *dsbcg_last_error(void) { return g_err.c_str(); }

int dsbcg_profile_enable(dsbcg_handle h, int32_t enable) {
    if (!h) return fail(DSBCG_ERR_ARG, "NULL handle");
    HIPCHK(prof_flush(h));
    for (int k = 0; k < kProfClasses; ++k) {
        h->prof_ms[k] = 0;
        h->prof_bytes[k] = 0;
        h->prof_launches[k] = 0;
    }
    h->prof = enable != 0;
    return DSBCG_OK;
}

int dsbcg_profile_select(dsbcg_handle h, uint32_t class_mask) {
    if (!h) return fail(DSBCG_ERR_ARG, "NULL handle");
    h->prof_mask = class_mask;
    return DSBCG_OK;
}

int dsbcg_profile_read(dsbcg_handle h, int32_t kclass, double *ms, int64_t *launches,
                       double *bytes) {
    if (!h) return fail(DSBCG_ERR_ARG, "NULL handle");
    if (kclass < 0 || kclass >= kProfClasses) return fail(DSBCG_ERR_ARG, "no such kernel class");
    HIPCHK(prof_flush(h));
    if (ms) *ms = h->prof_ms[kclass];
    if (launches) *launches = h->prof_launches[kclass];
    if (bytes) *bytes = h->prof_bytes[kclass];
    return DSBCG_OK;
}

const char *dsbcg_profile_name(int32_t kclass) {
    if (kclass < 0 || kclass >= kProfClasses) return nullptr;
    return kProfNames[kclass];
}

int dsbcg_create(const int32_t *L, dsbcg_handle *out) {
    if (!out) return fail(DSBCG_ERR_ARG, "out is NULL");
    *out = nullptr;
    CHK(validate_geom(L));
    dsbcg_ctx *h = new (std::nothrow) dsbcg_ctx();
    if (!h) return fail(DSBCG_ERR_OOM, "host allocation failed");
    for (int d = 0; d < 4; ++d) h->g.L[d] = L[d];
    h->g.V = L[0] * L[1] * L[2] * L[3];
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return fail(DSBCG_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    // the workspace of dsbcg_apply_A_noalloc on this device
    const int rc = noalloc_setup(h->device);
    if (rc != DSBCG_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return DSBCG_OK;
}

void dsbcg_destroy(dsbcg_handle h) { delete h; }

int dsbcg_neighbors(dsbcg_handle h, int32_t *host_out) {
    if (!h || !host_out) return fail(DSBCG_ERR_ARG, "NULL argument");
    int32_t *dev = nullptr;
    const size_t bytes = (size_t)h->g.V * 8 * sizeof(int32_t);
    HIPCHK(hipMalloc((void **)&dev, bytes));
    hipError_t e = neighbor_table(h->g, dev, nullptr);
    if (e == hipSuccess) e = hipMemcpy(host_out, dev, bytes, hipMemcpyDeviceToHost);
    (void)hipFree(dev);
    HIPCHK(e);
    return DSBCG_OK;
}

int dsbcg_stage_links(dsbcg_handle h, const void *U, dsbcg_stream stream) {
    if (!h || !U) return fail(DSBCG_ERR_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    CHK(ensure_common(h));
    h->links_staged = false;
    CHK(check_finite_links(h, U, st));
    CHK(prepare_links(h, U, true, st));
    CHK(prepare_links(h, U, false, st));
    HIPCHK(hipStreamSynchronize(st));
    h->links_staged = true;
    return DSBCG_OK;
}

int dsbcg_apply_D(dsbcg_handle h, const void *U, double kappa, const void *X, void *Y, int32_t m,
                  int32_t dagger, dsbcg_stream stream) {
    CHK(check_field_args(h, U, X, Y, m, kappa));
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = 12 * (int64_t)h->g.V;
    CHK(ensure_ws(h, h->Xin, (size_t)n * m * sizeof(zd)));
    CHK(use_links(h, U, false, false, st));
    CHK(copy(h, m, api(X, m), cm(h->Xin.p, n, true), false, st));
    // the pass writes the caller's layout directly
    CHK(stencil(h, true, h->Ul64.p, kappa, h->Xin.p, nullptr, m, dagger != 0, st, Y));
    return DSBCG_OK;
}

int dsbcg_apply_A(dsbcg_handle h, const void *U, double kappa, const void *X, void *Y, int32_t m,
                  int32_t precision, dsbcg_stream stream) {
    CHK(check_field_args(h, U, X, Y, m, kappa));
    if (precision != DSBCG_FP64 && precision != DSBCG_FP32_RELIABLE)
        return fail(DSBCG_ERR_ARG, "unknown precision");
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = precision == DSBCG_FP64;
    const int64_t n = 12 * (int64_t)h->g.V;
    const size_t esz = f64 ? sizeof(zd) : sizeof(zf);
    CHK(ensure_ws(h, h->Xin, (size_t)n * m * esz));
    CHK(ensure_ws(h, h->T, (size_t)n * m * esz));
    if (U) {
        // only the precision this call needs
        h->links_staged = false;
        CHK(prepare_links(h, U, f64, st));
    } else {
        CHK(use_links(h, U, false, false, st));
    }
    CHK(copy(h, m, api(X, m), cm(h->Xin.p, n, f64), false, st));
    // D X column-major, then D^H of it straight into the caller's layout
    const void *Ul = f64 ? h->Ul64.p : h->Ul32.p;
    CHK(stencil(h, f64, Ul, kappa, h->Xin.p, h->T.p, m, false, st));
    CHK(stencil(h, f64, Ul, kappa, h->T.p, nullptr, m, true, st, Y));
    return DSBCG_OK;
}

}  // extern "C"

namespace {

// Validated solve of (sigma_j I + A) X_j = B_j, B_j = B + j * bstride
// (bstride = 0: one B for every shift), followed by the FP64 true residuals
// and, for shifts that miss tol, FP64 re-solves of their residual blocks.
// Argument checks shared by the solve entry points; resolves the defaults of
// the options into *o.
int solve_args(dsbcg_handle h, const void *U, const void *B, int32_t m, const double *sigma, int32_t s,
               double tol, double kappa, const void *X, const dsbcg_opts *opts, dsbcg_opts *o) {
    if (!h || !B || !sigma || !X) return fail(DSBCG_ERR_ARG, "NULL argument");
    if (!U && !h->links_staged) return fail(DSBCG_ERR_ARG, "U is NULL and no links are staged on the handle");
    if (m < 1 || m > DSBCG_MAX_RHS) return fail(DSBCG_ERR_ARG, "m out of range");
    if (s < 1 || s > DSBCG_MAX_SHIFTS) return fail(DSBCG_ERR_ARG, "s out of range");
    if (!(tol > 0) || !std::isfinite(tol)) return fail(DSBCG_ERR_ARG, "tol must be > 0");
    if (!std::isfinite(kappa)) return fail(DSBCG_ERR_ARG, "kappa not finite");
    for (int j = 0; j < s; ++j)
        if (!std::isfinite(sigma[j])) return fail(DSBCG_ERR_ARG, "sigma not finite");
    dsbcg_default_opts(o);
    if (opts) *o = *opts;
    if (o->precision != DSBCG_FP64 && o->precision != DSBCG_FP32_RELIABLE)
        return fail(DSBCG_ERR_ARG, "unknown precision");
    if (o->window < 0) return fail(DSBCG_ERR_ARG, "window must be >= 0");
    if (o->tau_B < 0) o->tau_B = 0.1 * tol;
    if (o->tau_W < 0) o->tau_W = 1e-12;
    if (o->max_iters < 1) o->max_iters = 1;
    if (o->switch_at < 0) o->switch_at = std::min(1e-2, 1e5 * tol);
    return DSBCG_OK;
}

void fill_stats(dsbcg_stats *stats, const SolveStats &stt, const double *tr, int s, int m, double main_max) {
    if (!stats) return;
    double *est = stats->est_relres, *tru = stats->true_relres;
    if (est) std::copy(stt.est, stt.est + (size_t)s * m, est);
    if (tru) std::copy(tr, tr + (size_t)s * m, tru);
    stats->block_iters = stt.block_iters;
    stats->rank0 = stt.rank0;
    stats->deflations = stt.deflations;
    stats->reliable_updates = stt.reliable_updates;
    stats->refine_iters = stt.refine_iters;
    stats->final_width = stt.final_width;
    stats->switch_iter = stt.switch_iter;
    stats->qr2_skipped = stt.qr2_skipped;
    stats->qr_redone = stt.qr_redone;
    stats->main_relres_max = main_max;
    stats->mvms = stt.mvms;
    stats->mvms_vector = stt.mvms_vector;
    if (stats->frozen_at)
        for (size_t k = 0; k < (size_t)s * m; ++k)
            stats->frozen_at[k] = k < stt.frozen_at.size() ? stt.frozen_at[k] : 0;
    if (stats->widths)
        for (int32_t k = 0; k < stats->widths_len; ++k)
            stats->widths[k] = k < (int32_t)stt.widths.size() ? stt.widths[k] : 0;
    if (stats->est_history)
        for (int32_t k = 0; k < stats->widths_len; ++k)
            stats->est_history[k] = k < (int32_t)stt.est_hist.size() ? stt.est_hist[k] : 0.0;
}

int solve_checked(dsbcg_handle h, const void *U, double kappa, const void *B, int64_t bstride,
                  int32_t m, const double *sigma, int32_t s, double tol, const dsbcg_opts *opts,
                  void *X, dsbcg_stats *stats, hipStream_t st) {
    dsbcg_opts o;
    CHK(solve_args(h, U, B, m, sigma, s, tol, kappa, X, opts, &o));
    const int64_t n = 12 * (int64_t)h->g.V;

    CHK(ensure_common(h));
    CHK(use_links(h, U, o.precision == DSBCG_FP32_RELIABLE, true, st));

    SolveStats stt;
    double main_max = 0.0;
    int status = solve_core(h, kappa, B, bstride, m, sigma, s, tol, o, o.switch_at, X, stt, st, nullptr);
    bool fallback = false;
    if (status == DSBCG_ERR_ARG && bstride != 0 && stt.rank0 == 0) {
        // the blocks span more than 16 directions: one block solve per shift
        fallback = true;
        stt = SolveStats();
        status = DSBCG_OK;
        for (int j = 0; j < s && status == DSBCG_OK; ++j) {
            SolveStats one;
            status = solve_core(h, kappa, (const zd *)B + (int64_t)j * bstride, 0, m, &sigma[j], 1,
                                tol, o, o.switch_at, (zd *)X + (int64_t)j * n * m, one, st, nullptr);
            stt.block_iters += one.block_iters;
            stt.mvms += one.mvms;
            stt.reliable_updates += one.reliable_updates;
            stt.qr2_skipped += one.qr2_skipped;
            stt.qr_redone += one.qr_redone;
            stt.deflations += one.deflations;
            stt.rank0 = std::max(stt.rank0, one.rank0);
            stt.mvms_vector = std::max(stt.mvms_vector, one.mvms_vector);
            stt.frozen_at.resize((size_t)s * m, 0);
            for (int l = 0; l < m; ++l) {
                stt.est[j * m + l] = one.est[l];
                stt.frozen_at[(size_t)j * m + l] = one.frozen_at[l];
            }
        }
    }
    if (status != DSBCG_OK && status != DSBCG_ERR_NOT_CONVERGED) return status;

    std::vector<double> tr((size_t)s * m, 0.0);
    const bool want_true = (stats && stats->true_relres) || o.refine;
    if (want_true && status == DSBCG_OK) {
        // the iterates and the right-hand sides are still column-major in
        // h->X and h->Bint after one block solve over all shifts (not after
        // the per-shift fallback)
        const zd *xcm = !fallback ? (const zd *)h->X.p : nullptr;
        const zd *bcm = !fallback ? (const zd *)h->Bint.p : nullptr;
        CHK(true_residuals(h, st, kappa, B, bstride, X, m, sigma, s, tr.data(), -1, nullptr, xcm, bcm));
        for (double v : tr) main_max = std::max(main_max, v);
        for (int round = 0; o.refine && o.fixed_iters <= 0 && round < 2; ++round) {
            bool any = false;
            for (int j = 0; j < s; ++j) {
                double worst = 0.0;
                for (int l = 0; l < m; ++l) worst = std::max(worst, tr[j * m + l]);
                if (worst <= tol) continue;
                any = true;
                // residual block R_j, then (sigma_j + A) E = R_j and X_j += E.  The
                // first round of the FP32 form solves with FP32 vectors from the
                // start: it only has to reduce R_j by a small factor, far above
                // the FP32 residual gap; a second round runs in FP64.
                CHK(ensure_ws(h, h->Rres, (size_t)n * m * sizeof(zd)));
                CHK(ensure_ws(h, h->Xref, (size_t)n * m * sizeof(zd)));
                std::vector<double> tmp((size_t)s * m);
                CHK(true_residuals(h, st, kappa, B, bstride, X, m, sigma, s, tmp.data(), j, h->Rres.p));
                double ratio = 1e300;
                for (int l = 0; l < m; ++l)
                    if (tr[j * m + l] > 0) ratio = std::min(ratio, 1.0 / tr[j * m + l]);
                dsbcg_opts ro = o;
                const bool r32 = o.precision == DSBCG_FP32_RELIABLE && round == 0;
                ro.precision = r32 ? DSBCG_FP32_RELIABLE : DSBCG_FP64;
                ro.fixed_iters = 0;
                ro.tau_B = 0.1 * tol;
                SolveStats rs;
                const double rtol = std::max(0.5 * tol * ratio, 1e-15);
                int rc = solve_core(h, kappa, h->Rres.p, 0, m, &sigma[j], 1, rtol, ro, r32 ? 2.0 : 0.0, h->Xref.p,
                                    rs, st, nullptr);
                if (rc != DSBCG_OK && rc != DSBCG_ERR_NOT_CONVERGED) return rc;
                stt.refine_iters += rs.block_iters;
                stt.mvms += rs.mvms;
                CHK(copy(h, m, api(h->Xref.p, m), api((zd *)X + (int64_t)j * n * m, m), true, st));
            }
            if (!any) break;
            CHK(true_residuals(h, st, kappa, B, bstride, X, m, sigma, s, tr.data(), -1, nullptr));
        }
        double worst = 0.0;
        for (double v : tr) worst = std::max(worst, v);
        if (worst > tol && o.fixed_iters <= 0)
            status = fail(DSBCG_ERR_NOT_CONVERGED,
                          "true relative residual " + std::to_string(worst) + " above tol after refinement");
    }
    fill_stats(stats, stt, tr.data(), s, m, main_max);
    return status;
}

}  // namespace

extern "C" {

// Releases the solve workspace on every return of a solve entry point unless
// the caller asked to keep it (opts->keep_workspace).
struct WorkspaceScope {
    dsbcg_ctx *h;
    bool keep;
    WorkspaceScope(dsbcg_ctx *hh, const dsbcg_opts *opts) : h(hh), keep(!opts || opts->keep_workspace) {}
    ~WorkspaceScope() {
        if (h && !keep) release_workspace(h);
    }
};

int dsbcg_solve(dsbcg_handle h, const void *U, double kappa, const void *B, int32_t m,
                const double *sigma, int32_t s, double tol, const dsbcg_opts *opts, void *X,
                dsbcg_stats *stats, dsbcg_stream stream) {
    WorkspaceScope ws(h, opts);
    return solve_checked(h, U, kappa, B, 0, m, sigma, s, tol, opts, X, stats, (hipStream_t)stream);
}

int dsbcg_release_workspace(dsbcg_handle h) {
    if (!h) return fail(DSBCG_ERR_ARG, "NULL handle");
    HIPCHK(hipDeviceSynchronize());
    release_workspace(h);
    return DSBCG_OK;
}

int dsbcg_solve_rational(dsbcg_handle h, const void *U, double kappa, const void *B, int32_t m,
                         const double *sigma, const double *coef, int32_t s, double c0, double tol,
                         const dsbcg_opts *opts, void *Y, dsbcg_stats *stats, dsbcg_stream stream) {
    hipStream_t st = (hipStream_t)stream;
    WorkspaceScope ws(h, opts);
    dsbcg_opts o;
    CHK(solve_args(h, U, B, m, sigma, s, tol, kappa, Y, opts, &o));
    if (!coef) return fail(DSBCG_ERR_ARG, "NULL argument");
    if (!std::isfinite(c0)) return fail(DSBCG_ERR_ARG, "c0 not finite");
    for (int j = 0; j < s; ++j)
        if (!std::isfinite(coef[j])) return fail(DSBCG_ERR_ARG, "coefficient not finite");
    if (Y == B) return fail(DSBCG_ERR_ARG, "Y must not alias B");
    const int64_t n = 12 * (int64_t)h->g.V;
    CHK(ensure_common(h));
    if (o.precision == DSBCG_FP32_RELIABLE) {
        // the checked solve (FP64 true residuals, re-solves) into workspace,
        // then Y = c0 B + sum_j c_j X_j
        CHK(ensure_ws(h, h->Xrat, (size_t)n * m * s * sizeof(zd)));
        const int status = solve_checked(h, U, kappa, B, 0, m, sigma, s, tol, &o, h->Xrat.p, stats, st);
        if (status != DSBCG_OK && status != DSBCG_ERR_NOT_CONVERGED) return status;
        PROF_LAUNCH(h, kProfConvert, copy_bytes(h->g.V, m, 16, 16, false), st,
                    copy_field(h->g.V, m, api(B, m), api(Y, m), false, c0, st));
        for (int j = 0; j < s; ++j)
            PROF_LAUNCH(h, kProfConvert, copy_bytes(h->g.V, m, 16, 16, true), st,
                        copy_field(h->g.V, m, api((const zd *)h->Xrat.p + (int64_t)j * n * m, m), api(Y, m),
                                   true, coef[j], st));
        HIPCHK(hipStreamSynchronize(st));
        return status;
    }
    CHK(use_links(h, U, false, true, st));
    SolveStats stt;
    RatSpec rs{coef, c0, Y};
    const int status = solve_core(h, kappa, B, 0, m, sigma, s, tol, o, o.switch_at, nullptr, stt, st, &rs);
    if (status != DSBCG_OK && status != DSBCG_ERR_NOT_CONVERGED) return status;
    // no per-shift iterates, so no true residuals: reported as -1
    std::vector<double> tr((size_t)s * m, -1.0);
    fill_stats(stats, stt, tr.data(), s, m, -1.0);
    return status;
}

int dsbcg_solve_multi(dsbcg_handle h, const void *U, double kappa, const void *B, int32_t m,
                      const double *sigma, int32_t s, double tol, const dsbcg_opts *opts, void *X,
                      dsbcg_stats *stats, dsbcg_stream stream) {
    if (!h) return fail(DSBCG_ERR_ARG, "NULL handle");
    WorkspaceScope ws(h, opts);
    return solve_checked(h, U, kappa, B, 12 * (int64_t)h->g.V * m, m, sigma, s, tol, opts, X, stats,
                         (hipStream_t)stream);
}

int dsbcg_grad(dsbcg_handle h, const void *U, double kappa, const double *sigma, int32_t s, int32_t m,
               const void *X, const void *Lam, void *dU, void *dB, double *dsigma, dsbcg_stream stream) {
    if (!h || !sigma || !X || !Lam) return fail(DSBCG_ERR_ARG, "NULL argument");
    if (dU && !U && !h->links_staged)
        return fail(DSBCG_ERR_ARG, "U is NULL and no links are staged on the handle");
    if (m < 1 || m > DSBCG_MAX_RHS || s < 1 || s > DSBCG_MAX_SHIFTS)
        return fail(DSBCG_ERR_ARG, "m or s out of range");
    if (!std::isfinite(kappa)) return fail(DSBCG_ERR_ARG, "kappa not finite");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = 12 * (int64_t)h->g.V;
    const size_t blk = (size_t)n * m * sizeof(zd);
    CHK(ensure_common(h));
    CHK(ensure_ws(h, h->R0, blk));
    CHK(ensure_ws(h, h->R1, blk));
    CHK(ensure_ws(h, h->R2, blk));
    CHK(ensure_ws(h, h->R3, blk));
    if (dU) CHK(use_links(h, U, false, false, st));
    Ts ts{h, true, st, n};
    for (int j = 0; j < s; ++j) {
        const zd *Xj = (const zd *)X + (int64_t)j * n * m;
        const zd *Lj = (const zd *)Lam + (int64_t)j * n * m;
        // dL/dB = sum_j Lambda_j
        if (dB) CHK(copy(h, m, api(Lj, m), api(dB, m), j > 0, st));
        CHK(copy(h, m, api(Xj, m), cm(h->R0.p, n, true), false, st));
        CHK(copy(h, m, api(Lj, m), cm(h->R1.p, n, true), false, st));
        if (dsigma) {
            // dL/dsigma_j = -Re <Lambda_j, X_j>
            TsArgs a = ts_args(n);
            a.K = 1;
            a.X[0] = h->R0.p; a.bx[0] = m; a.C[0] = nullptr;
            a.bout = m;
            a.gram = 2; a.L = h->R1.p; a.bl = m;
            CHK(ts.run_reduce(a, m, 6));
            std::vector<zd> g(256);
            HIPCHK(hipMemcpyAsync(g.data(), red_slot(h, 6), 256 * sizeof(zd), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            double tr = 0.0;
            for (int l = 0; l < m; ++l) tr += g[l * 16 + l].x;
            dsigma[j] = -tr;
        }
        if (dU) {
            // dL/dU = -sum_j [ d Re <D X_j, D Lambda_j> + d Re <D Lambda_j, D X_j> ]
            CHK(stencil(h, true, h->Ul64.p, kappa, h->R0.p, h->R2.p, m, false, st));   // D X_j
            CHK(stencil(h, true, h->Ul64.p, kappa, h->R1.p, h->R3.p, m, false, st));   // D Lambda_j
            // algorithmic bytes: each field read once, dU written (and read
            // when accumulating)
            PROF_LAUNCH(h, kProfGrad, (double)h->g.V * (2.0 * 12 * m + 36.0 * (j ? 2 : 1)) * 16, st,
                        link_grad_apply(h->g, kappa, h->R2.p, h->R1.p, m, dU, j > 0, -1.0, st));
            PROF_LAUNCH(h, kProfGrad, (double)h->g.V * (2.0 * 12 * m + 72.0) * 16, st,
                        link_grad_apply(h->g, kappa, h->R3.p, h->R0.p, m, dU, true, -1.0, st));
        }
    }
    return DSBCG_OK;
}

int dsbcg_link_grad(dsbcg_handle h, double kappa, const void *Phi, const void *Psi, int32_t nvec,
                    void *dU, dsbcg_stream stream) {
    if (!h || !Phi || !Psi || !dU) return fail(DSBCG_ERR_ARG, "NULL argument");
    if (nvec < 1 || nvec > DSBCG_MAX_RHS * DSBCG_MAX_SHIFTS)
        return fail(DSBCG_ERR_ARG, "nvec out of range");
    if (!std::isfinite(kappa)) return fail(DSBCG_ERR_ARG, "kappa not finite");
    hipStream_t st = (hipStream_t)stream;
    const int64_t V = h->g.V;
    // the kernel reads both fields column-major; convert in chunks of <= 16 columns
    const int64_t n = 12 * V;
    const int chunk = std::min<int>(nvec, 16);
    CHK(ensure_ws(h, h->Xin, (size_t)n * chunk * sizeof(zd)));
    CHK(ensure_ws(h, h->Yout, (size_t)n * chunk * sizeof(zd)));
    for (int c0 = 0; c0 < nvec; c0 += chunk) {
        const int cols = std::min(chunk, nvec - c0);
        CHK(copy(h, cols, FieldDesc{const_cast<void *>(Phi), kApi, nvec, c0, true},
                 cm(h->Xin.p, n, true), false, st));
        CHK(copy(h, cols, FieldDesc{const_cast<void *>(Psi), kApi, nvec, c0, true},
                 cm(h->Yout.p, n, true), false, st));
        PROF_LAUNCH(h, kProfGrad, (double)V * (2.0 * 12 * cols + 36.0 * (c0 ? 2 : 1)) * 16, st,
                    link_grad_apply(h->g, kappa, h->Xin.p, h->Yout.p, cols, dU, c0 > 0, 1.0, st));
    }
    return DSBCG_OK;
}

}  // extern "C"

namespace dsbcg {

void handle_view(dsbcg_handle h, Geom *g, int *device, const void **ul64, const void **ul32) {
    *g = h->g;
    *device = h->device;
    *ul64 = h->links_staged ? h->Ul64.p : nullptr;
    *ul32 = h->links_staged ? h->Ul32.p : nullptr;
}

int set_error(int code, const char *msg) { return fail(code, msg); }

}  // namespace dsbcg
