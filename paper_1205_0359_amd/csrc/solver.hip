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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dsbcg.h"
#include "blas.hpp"
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

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

enum ProfClass {
    kProfStencil = 0,   // one Wilson D or D^H pass
    kProfBlock,         // tall-skinny combination / Gram kernels of the block step
    kProfShift,         // fused per-shift P_j / X_j update
    kProfSmall,         // small FP64 algebra and Gram reductions
    kProfConvert,       // layout conversions, widening, accumulation
    kProfClasses
};
const char *const kProfNames[kProfClasses] = {"wilson_stencil", "block_gram_update",
                                              "shift_update", "small_algebra", "convert"};

struct ProfRec {
    int cls;
    hipEvent_t a, b;
    double bytes;
};

struct dsbcg_ctx {
    Geom g{};
    int device = 0;
    bool lds_links = true;
    // kernel timing (dsbcg_profile_enable)
    bool prof = false;
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    double prof_ms[kProfClasses] = {};
    double prof_bytes[kProfClasses] = {};
    int64_t prof_launches[kProfClasses] = {};
    // workspace
    DevBuf U32, T, W, V[3], P[2], X, Bint, Q, wbuf, Rf64a, Rf64b, X32in;
    DevBuf V32[3], T32, W32, P32[2], Xlo, Rres, Xref;
    DevBuf partials, red, list, st, rep;
    StepReport *rep_host = nullptr;
    int32_t *list_host = nullptr;
    int nwg_max = 2048;

    ~dsbcg_ctx() {
        DevBuf *all[] = {&U32,   &T,     &W,     &V[0],  &V[1],   &V[2],   &P[0],     &P[1],
                         &X,     &Bint,  &Q,     &wbuf,  &Rf64a,  &Rf64b,  &X32in,    &V32[0],
                         &V32[1], &V32[2], &T32, &W32,   &P32[0], &P32[1], &Xlo,      &Rres,
                         &Xref,  &partials, &red, &list, &st,     &rep};
        for (DevBuf *b : all)
            if (b->p) (void)hipFree(b->p);
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

#define CHK(expr)                          \
    do {                                   \
        int rc_ = (expr);                  \
        if (rc_ != DSBCG_OK) return rc_;   \
    } while (0)

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

ProfToken prof_begin(dsbcg_ctx *h, hipStream_t st) {
    ProfToken t;
    if (!h->prof) return t;
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
        ProfToken tok_ = prof_begin((h), (st));               \
        HIPCHK(expr);                                         \
        HIPCHK(prof_end((h), tok_, (cls), (bytes), (st)));    \
    } while (0)

// algorithmic bytes of one Wilson pass on nb columns: read nb spinors and
// the links, write nb spinors
double stencil_bytes(const Geom &g, int nb, size_t esz) {
    return (double)g.V * (2.0 * 12 * nb + 36.0) * (double)esz;
}

double shift_bytes(const ShiftArgs &a, bool fp64) {
    // V_i row once; per shift: P_{j,i-1} row, P_{j,i} row, X_j row read and written
    double cols = a.b;
    for (int js = 0; js < a.nshift; ++js) cols += (a.first ? 0 : a.bp) + a.b + 2.0 * a.m;
    return cols * (double)a.nrows * (double)(fp64 ? sizeof(zd) : sizeof(zf));
}

double copy_bytes(int64_t V, int cols, size_t in_esz, size_t out_esz, bool accumulate) {
    return (double)V * 12 * cols * ((double)in_esz + (accumulate ? 2.0 : 1.0) * (double)out_esz);
}

int ensure_common(dsbcg_ctx *h) {
    CHK(ensure(h->partials, (size_t)h->nwg_max * 256 * sizeof(zd)));
    CHK(ensure(h->red, 8 * 256 * sizeof(zd)));
    CHK(ensure(h->list, 64 * sizeof(int32_t)));
    CHK(ensure(h->st, sizeof(SmallState)));
    CHK(ensure(h->rep, sizeof(StepReport)));
    if (!h->rep_host) HIPCHK(hipHostMalloc((void **)&h->rep_host, sizeof(StepReport), 0));
    if (!h->list_host) HIPCHK(hipHostMalloc((void **)&h->list_host, 64 * sizeof(int32_t), 0));
    return DSBCG_OK;
}

zd *red_slot(dsbcg_ctx *h, int k) { return (zd *)h->red.p + 256 * k; }

// Tall-skinny combination / Gram launch.  Returns the number of workgroups
// whose partials must be reduced.
struct Ts {
    dsbcg_ctx *h;
    bool fp64;
    hipStream_t st;
    int64_t nrows;

    int run(TsArgs a, int *nwg_out) {
        const int TR = fp64 ? 32 : 64;
        int64_t tiles = (nrows + TR - 1) / TR;
        int nwg = (int)std::min<int64_t>(tiles, h->nwg_max);
        if (nwg < 1) nwg = 1;
        int64_t per = (tiles + nwg - 1) / nwg;
        a.rows_per_wg = per * TR;
        nwg = (int)((nrows + a.rows_per_wg - 1) / a.rows_per_wg);
        if (nwg < 1) nwg = 1;
        a.nrows = nrows;
        a.partials = (zd *)h->partials.p;
        double per_row = 0;
        for (int k = 0; k < a.K; ++k) per_row += a.bx[k];
        if (a.out) per_row += a.bout;
        if (a.gram == 2) per_row += a.bl;
        const double bytes = per_row * (double)nrows * (fp64 ? sizeof(zd) : sizeof(zf));
        PROF_LAUNCH(h, kProfBlock, bytes, st, ts_run(fp64, a, nwg, st));
        if (nwg_out) *nwg_out = nwg;
        return DSBCG_OK;
    }
    // run + reduce of rows p < rows_used into red slot k
    int run_reduce(TsArgs a, int rows_used, int k) {
        int nwg = 0;
        CHK(run(a, &nwg));
        if (rows_used > 0)
            PROF_LAUNCH(h, kProfSmall, 0.0, st,
                        reduce_partials((zd *)h->partials.p, nwg, rows_used * 16, red_slot(h, k), st));
        return DSBCG_OK;
    }
};

TsArgs ts_args() {
    TsArgs a;
    memset(&a, 0, sizeof(a));
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

// Plane layout of an n x b block: element (x, c, r) at (c*V + x)*b + r.
inline int64_t plane_site(int b) { return b; }
inline int64_t plane_comp(const Geom &g, int b) { return (int64_t)g.V * b; }

// Y = A X on b columns, FP64 or FP32 data; X and Y in plane layout with
// leading dimension b, T scratch of the same shape.
int apply_A_plane(dsbcg_ctx *h, bool fp64, const void *U, double kappa, const void *X, void *T,
                  void *Y, int b, hipStream_t st) {
    const double bytes = stencil_bytes(h->g, b, fp64 ? sizeof(zd) : sizeof(zf));
    PROF_LAUNCH(h, kProfStencil, bytes, st,
                wilson_apply(h->g, fp64, U, kappa, X, plane_site(b), plane_comp(h->g, b), T,
                             plane_site(b), plane_comp(h->g, b), b, false, h->lds_links, st));
    PROF_LAUNCH(h, kProfStencil, bytes, st,
                wilson_apply(h->g, fp64, U, kappa, T, plane_site(b), plane_comp(h->g, b), Y,
                             plane_site(b), plane_comp(h->g, b), b, true, h->lds_links, st));
    return DSBCG_OK;
}

struct SolveCtx {
    dsbcg_ctx *h;
    hipStream_t st;
    bool fp64;          // data precision of the iteration
    size_t esz;         // bytes per complex element of the iteration
    int64_t V, n;
    int m, s;
    const void *Ulinks; // links in the iteration precision
    double kappa;
    double tol;
    dsbcg_opts o;
};

struct SolveStats {
    int32_t block_iters = 0, rank0 = 0, deflations = 0, reliable_updates = 0, refine_iters = 0;
    int32_t final_width = 0, switch_iter = 0;
    int64_t mvms = 0;
    double est[kS * kS] = {};
};

// Initial deflated QR of B (plane layout FP64, ld m): CGS2 column by column.
// Leaves V_1 (iteration precision, ld m1) in V[0] and rho in the small state.
int initial_qr(SolveCtx &c, int *m1_out) {
    dsbcg_ctx *h = c.h;
    const int m = c.m;
    Ts ts{h, true, c.st, c.n};
    SmallState *S = stp(h);
    StepReport *rep = repp(h);
    // ||b_l|| from the diagonal of B^H B
    {
        TsArgs a = ts_args();
        a.K = 1;
        a.X[0] = h->Bint.p; a.ldx[0] = m; a.bx[0] = m; a.C[0] = nullptr;
        a.bout = m;
        a.gram = 1;
        CHK(ts.run_reduce(a, m, 0));
        PROF_LAUNCH(c.h, kProfSmall, 0.0, c.st, small_bnorms(S, rep, red_slot(h, 0), m, c.st));
    }
    int k = 0;
    zd *Qp = (zd *)h->Q.p;
    zd *Bp = (zd *)h->Bint.p;
    zd *wp = (zd *)h->wbuf.p;
    for (int l = 0; l < m; ++l) {
        if (k > 0) {
            // c1 = Q^H b_l
            TsArgs a = ts_args();
            a.K = 1;
            a.X[0] = Bp + l; a.ldx[0] = m; a.bx[0] = 1; a.C[0] = nullptr;
            a.bout = 1;
            a.gram = 2; a.L = Qp; a.ldl = m; a.bl = k;
            CHK(ts.run_reduce(a, k, 1));
            PROF_LAUNCH(c.h, kProfSmall, 0.0, c.st, small_neg_column(S, 0, red_slot(h, 1), k, c.st));
            // w = b_l - Q c1, c2 = Q^H w
            a = ts_args();
            a.K = 2;
            a.X[0] = Bp + l; a.ldx[0] = m; a.bx[0] = 1; a.C[0] = nullptr;
            a.X[1] = Qp; a.ldx[1] = m; a.bx[1] = k; a.C[1] = coef_slot(h, 0);
            a.bout = 1;
            a.out = wp; a.ldo = 1;
            a.gram = 2; a.L = Qp; a.ldl = m; a.bl = k;
            CHK(ts.run_reduce(a, k, 2));
            PROF_LAUNCH(c.h, kProfSmall, 0.0, c.st, small_neg_column(S, 1, red_slot(h, 2), k, c.st));
            // w = w - Q c2, ||w||^2
            a = ts_args();
            a.K = 2;
            a.X[0] = wp; a.ldx[0] = 1; a.bx[0] = 1; a.C[0] = nullptr;
            a.X[1] = Qp; a.ldx[1] = m; a.bx[1] = k; a.C[1] = coef_slot(h, 1);
            a.bout = 1;
            a.out = wp; a.ldo = 1;
            a.gram = 1;
            CHK(ts.run_reduce(a, 1, 3));
            PROF_LAUNCH(c.h, kProfSmall, 0.0, c.st, small_cgs_decide(S, rep, red_slot(h, 1), red_slot(h, 2), red_slot(h, 3), k, l,
                                    c.o.tau_B, c.st));
        } else {
            TsArgs a = ts_args();
            a.K = 1;
            a.X[0] = Bp + l; a.ldx[0] = m; a.bx[0] = 1; a.C[0] = nullptr;
            a.bout = 1;
            a.out = wp; a.ldo = 1;
            a.gram = 1;
            CHK(ts.run_reduce(a, 1, 3));
            PROF_LAUNCH(c.h, kProfSmall, 0.0, c.st, small_cgs_decide(S, rep, nullptr, nullptr, red_slot(h, 3), 0, l, c.o.tau_B, c.st));
        }
        CHK(read_report(h, c.st));
        if (h->rep_host->flags & kFlagNonFinite)
            return fail(DSBCG_ERR_NOT_HPD, "B holds non-finite values");
        if (h->rep_host->scalar[1] > 0.5) {
            // Q[:, k] = w / ||w||
            TsArgs a = ts_args();
            a.K = 1;
            a.X[0] = wp; a.ldx[0] = 1; a.bx[0] = 1; a.C[0] = coef_slot(h, 3);
            a.bout = 1;
            a.out = Qp + k; a.ldo = m;
            CHK(ts.run(a, nullptr));
            ++k;
        }
    }
    // V_1 = Q[:, :k] with leading dimension k, in the iteration precision
    if (k > 0)
        PROF_LAUNCH(c.h, kProfConvert, copy_bytes(c.V, k, (true) ? 16 : 8, (c.fp64) ? 16 : 8, false), c.st, copy_field(true, c.fp64, c.V, k, Qp, m, kPlane, 0, h->V[0].p, k, kPlane, false, 1.0,
                          c.st));
    *m1_out = k;
    return DSBCG_OK;
}

int check_finite_links(dsbcg_ctx *h, const void *U, hipStream_t st) {
    StepReport *rep = repp(h);
    HIPCHK(hipMemsetAsync(&rep->flags, 0, sizeof(int32_t), st));
    PROF_LAUNCH(h, kProfConvert, (double)h->g.V * 72 * 8, st, find_nonfinite((const double *)U, (int64_t)h->g.V * 72, &rep->flags, st));
    int32_t flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, &rep->flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (flag) return fail(DSBCG_ERR_NOT_HPD, "U holds non-finite values");
    return DSBCG_OK;
}

// True relative residuals ||b_l - (sigma_j + A) x_{l,j}|| / ||b_l|| in FP64 for
// every shift; B and X in API layout.  With keep_j >= 0 the residual block of
// that shift is also stored (API layout) in Rkeep.
int true_residuals(dsbcg_ctx *h, hipStream_t st, const void *U64, double kappa, const void *Bapi,
                   const void *Xapi, int m, const double *sigma, int s, double *out, int keep_j,
                   void *Rkeep) {
    const int64_t n = 12 * (int64_t)h->g.V;
    const int64_t api_site = 12 * (int64_t)m, api_comp = m;
    CHK(ensure_common(h));
    CHK(ensure(h->Rf64a, (size_t)n * m * sizeof(zd)));
    CHK(ensure(h->Rf64b, (size_t)n * m * sizeof(zd)));
    Ts ts{h, true, st, n};
    std::vector<double> bn(m);
    {
        TsArgs a = ts_args();
        a.K = 1;
        a.X[0] = Bapi; a.ldx[0] = m; a.bx[0] = m; a.C[0] = nullptr;
        a.bout = m;
        a.gram = 1;
        CHK(ts.run_reduce(a, m, 4));
        std::vector<zd> g(256);
        HIPCHK(hipMemcpyAsync(g.data(), red_slot(h, 4), 256 * sizeof(zd), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int l = 0; l < m; ++l) bn[l] = std::sqrt(std::max(g[l * 16 + l].x, 0.0));
    }
    std::vector<zd> cf(512, mk<double>(0, 0));
    for (int j = 0; j < s; ++j) {
        if (keep_j >= 0 && j != keep_j) continue;
        const zd *Xj = (const zd *)Xapi + (int64_t)j * n * m;
        const double sb = stencil_bytes(h->g, m, sizeof(zd));
        PROF_LAUNCH(h, kProfStencil, sb, st,
                    wilson_apply(h->g, true, U64, kappa, Xj, api_site, api_comp, h->Rf64a.p,
                                 api_site, api_comp, m, false, h->lds_links, st));
        PROF_LAUNCH(h, kProfStencil, sb, st,
                    wilson_apply(h->g, true, U64, kappa, h->Rf64a.p, api_site, api_comp,
                                 h->Rf64b.p, api_site, api_comp, m, true, h->lds_links, st));
        TsArgs a = ts_args();
        a.K = 3;
        a.X[0] = Bapi; a.ldx[0] = m; a.bx[0] = m; a.C[0] = nullptr;
        a.X[1] = Xj; a.ldx[1] = m; a.bx[1] = m; a.C[1] = coef_slot(h, 2);
        a.X[2] = h->Rf64b.p; a.ldx[2] = m; a.bx[2] = m; a.C[2] = coef_slot(h, 3);
        a.bout = m;
        a.gram = 1;
        if (keep_j >= 0) {
            a.out = Rkeep;
            a.ldo = m;
        }
        // coefficient matrices -sigma_j I and -I
        for (int l = 0; l < m; ++l) {
            cf[l * 16 + l] = mk<double>(-sigma[j], 0);
            cf[256 + l * 16 + l] = mk<double>(-1.0, 0);
        }
        HIPCHK(hipMemcpyAsync((void *)coef_slot(h, 2), cf.data(), 512 * sizeof(zd),
                              hipMemcpyHostToDevice, st));
        CHK(ts.run_reduce(a, m, 5));
        std::vector<zd> g(256);
        HIPCHK(hipMemcpyAsync(g.data(), red_slot(h, 5), 256 * sizeof(zd), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int l = 0; l < m; ++l) {
            const double r = std::sqrt(std::max(g[l * 16 + l].x, 0.0));
            out[j * m + l] = bn[l] > 0 ? r / bn[l] : 0.0;
        }
    }
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
    o->tau_B = -1.0;  // resolved to 0.1 * tol
    o->tau_W = -1.0;  // resolved to 1e-12
    o->refine = 1;
    o->freeze = 1;
    o->switch_at = -1.0;  // resolved to min(1e-2, 1e6 * tol)
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
    const char *v = getenv("DSBCG_LDS_LINKS");
    if (v && v[0] == '0') h->lds_links = false;
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

int dsbcg_apply_D(dsbcg_handle h, const void *U, double kappa, const void *X, void *Y, int32_t m,
                  int32_t dagger, dsbcg_stream stream) {
    if (!h || !U || !X || !Y) return fail(DSBCG_ERR_ARG, "NULL argument");
    if (m < 1 || m > DSBCG_MAX_RHS) return fail(DSBCG_ERR_ARG, "m out of range");
    if (!std::isfinite(kappa)) return fail(DSBCG_ERR_ARG, "kappa not finite");
    if (X == Y) return fail(DSBCG_ERR_ARG, "Y must not alias X");
    hipStream_t st = (hipStream_t)stream;
    PROF_LAUNCH(h, kProfStencil, stencil_bytes(h->g, m, sizeof(zd)), st,
                wilson_apply(h->g, true, U, kappa, X, 12 * (int64_t)m, m, Y, 12 * (int64_t)m, m, m,
                             dagger != 0, h->lds_links, st));
    return DSBCG_OK;
}

int dsbcg_apply_A(dsbcg_handle h, const void *U, double kappa, const void *X, void *Y, int32_t m,
                  int32_t precision, dsbcg_stream stream) {
    if (!h || !U || !X || !Y) return fail(DSBCG_ERR_ARG, "NULL argument");
    if (m < 1 || m > DSBCG_MAX_RHS) return fail(DSBCG_ERR_ARG, "m out of range");
    if (!std::isfinite(kappa)) return fail(DSBCG_ERR_ARG, "kappa not finite");
    if (X == Y) return fail(DSBCG_ERR_ARG, "Y must not alias X");
    if (precision != DSBCG_FP64 && precision != DSBCG_FP32_RELIABLE)
        return fail(DSBCG_ERR_ARG, "unknown precision");
    hipStream_t st = (hipStream_t)stream;
    const int64_t V = h->g.V, n = 12 * V;
    const int64_t api_site = 12 * (int64_t)m, api_comp = m;
    if (precision == DSBCG_FP64) {
        CHK(ensure(h->T, (size_t)n * m * sizeof(zd)));
        const double sb = stencil_bytes(h->g, m, sizeof(zd));
        PROF_LAUNCH(h, kProfStencil, sb, st,
                    wilson_apply(h->g, true, U, kappa, X, api_site, api_comp, h->T.p, api_site,
                                 api_comp, m, false, h->lds_links, st));
        PROF_LAUNCH(h, kProfStencil, sb, st,
                    wilson_apply(h->g, true, U, kappa, h->T.p, api_site, api_comp, Y, api_site,
                                 api_comp, m, true, h->lds_links, st));
        return DSBCG_OK;
    }
    // FP32: round links and X, apply in FP32 (plane layout), widen the result
    CHK(ensure(h->U32, (size_t)V * 36 * sizeof(zf)));
    CHK(ensure(h->X32in, (size_t)n * m * sizeof(zf)));
    CHK(ensure(h->T, (size_t)n * m * sizeof(zf)));
    CHK(ensure(h->W, (size_t)n * m * sizeof(zf)));
    // links: [V][4][3][3] has the same shape as a [V*3][.][12] field... copy flat
    PROF_LAUNCH(h, kProfConvert, copy_bytes(V * 3, 1, (true) ? 16 : 8, (false) ? 16 : 8, false), st, copy_field(true, false, V * 3, 1, U, 1, kPlane, 0, h->U32.p, 1, kPlane, false, 1.0, st));
    PROF_LAUNCH(h, kProfConvert, copy_bytes(V, m, (true) ? 16 : 8, (false) ? 16 : 8, false), st, copy_field(true, false, V, m, X, m, kApi, 0, h->X32in.p, m, kPlane, false, 1.0, st));
    CHK(apply_A_plane(h, false, h->U32.p, kappa, h->X32in.p, h->T.p, h->W.p, m, st));
    PROF_LAUNCH(h, kProfConvert, copy_bytes(V, m, (false) ? 16 : 8, (true) ? 16 : 8, false), st, copy_field(false, true, V, m, h->W.p, m, kPlane, 0, Y, m, kApi, false, 1.0, st));
    return DSBCG_OK;
}

}  // extern "C"

namespace {

// Buffers of one working precision.
struct WorkSet {
    void *V[3];
    void *T, *W;
    void *P[2];
    void *X;            // solution accumulator, plane layout, leading dimension m
    const void *U;      // links
    const void *N, *M;  // per-shift coefficients in this precision
    bool fp64;
    size_t esz;
};

int convert_block(dsbcg_ctx *h, int64_t V, int cols, const void *in, bool in64, void *out, bool out64,
                  hipStream_t st) {
    if (cols <= 0) return DSBCG_OK;
    PROF_LAUNCH(h, kProfConvert, copy_bytes(V, cols, in64 ? 16 : 8, out64 ? 16 : 8, false), st,
                copy_field(in64, out64, V, cols, in, cols, kPlane, 0, out, cols, kPlane, false, 1.0, st));
    return DSBCG_OK;
}

// The DSBlockCG iteration.  FP64 form: every vector in FP64.  FP32 form: the
// iteration starts in FP64 and continues with FP32 vectors once every active
// estimate is <= switch_at; from then on X_j = X_hi + X_lo with X_lo in FP32,
// flushed into the FP64 X_hi every ru_interval steps and at the end.
// Writes the iterates to Xapi ([s][V][4][3][m], FP64).
int solve_core(dsbcg_ctx *h, const void *U, double kappa, const void *B, int m, const double *sigma,
               int s, double tol, const dsbcg_opts &o, double switch_at, void *Xapi,
               SolveStats &stt, hipStream_t st) {
    SolveCtx c;
    c.h = h;
    c.st = st;
    c.fp64 = true;
    c.esz = sizeof(zd);
    c.V = h->g.V;
    c.n = 12 * c.V;
    c.m = m;
    c.s = s;
    c.kappa = kappa;
    c.tol = tol;
    c.o = o;
    c.Ulinks = U;
    const int64_t n = c.n;
    const bool form32 = o.precision == DSBCG_FP32_RELIABLE;

    CHK(ensure_common(h));
    CHK(ensure(h->Bint, (size_t)n * m * sizeof(zd)));
    CHK(ensure(h->Q, (size_t)n * m * sizeof(zd)));
    CHK(ensure(h->wbuf, (size_t)n * sizeof(zd)));
    CHK(ensure(h->V[0], (size_t)n * m * sizeof(zd)));
    CHK(ensure(h->X, (size_t)n * m * s * sizeof(zd)));

    SmallState *S = stp(h);
    StepReport *rep = repp(h);
    CHK(check_finite_links(h, U, st));
    HIPCHK(hipMemsetAsync(rep, 0, sizeof(StepReport), st));
    HIPCHK(hipMemsetAsync(h->X.p, 0, (size_t)n * m * s * sizeof(zd), st));
    PROF_LAUNCH(h, kProfConvert, copy_bytes(c.V, m, 16, 16, false), st,
                copy_field(true, true, c.V, m, B, m, kApi, 0, h->Bint.p, m, kPlane, false, 1.0, st));

    int m1 = 0;
    CHK(initial_qr(c, &m1));
    stt.rank0 = m1;
    PROF_LAUNCH(h, kProfSmall, 0.0, st,
                small_init_shifts(S, rep, m1, m, s, sigma, o.freeze, tol, st));
    CHK(read_report(h, st));

    // widths never exceed m1 after the initial deflation
    const int wmax = std::max(m1, 1);
    const size_t b64 = (size_t)n * wmax * sizeof(zd), b32 = (size_t)n * wmax * sizeof(zf);
    for (int k = 0; k < 3; ++k) CHK(ensure(h->V[k], std::max(b64, (size_t)n * m * sizeof(zd))));
    CHK(ensure(h->T, (size_t)n * m * sizeof(zd)));
    CHK(ensure(h->W, (size_t)n * m * sizeof(zd)));
    CHK(ensure(h->P[0], b64 * s));
    CHK(ensure(h->P[1], b64 * s));
    WorkSet w64{{h->V[0].p, h->V[1].p, h->V[2].p}, h->T.p, h->W.p, {h->P[0].p, h->P[1].p}, h->X.p,
                U, S->N, S->M, true, sizeof(zd)};
    WorkSet w32{};
    if (form32) {
        CHK(ensure(h->U32, (size_t)c.V * 36 * sizeof(zf)));
        for (int k = 0; k < 3; ++k) CHK(ensure(h->V32[k], b32));
        CHK(ensure(h->T32, b32));
        CHK(ensure(h->W32, b32));
        CHK(ensure(h->P32[0], b32 * s));
        CHK(ensure(h->P32[1], b32 * s));
        CHK(ensure(h->Xlo, (size_t)n * m * s * sizeof(zf)));
        PROF_LAUNCH(h, kProfConvert, copy_bytes(c.V * 3, 1, 16, 8, false), st,
                    copy_field(true, false, c.V * 3, 1, U, 1, kPlane, 0, h->U32.p, 1, kPlane, false, 1.0, st));
        w32 = WorkSet{{h->V32[0].p, h->V32[1].p, h->V32[2].p}, h->T32.p, h->W32.p,
                      {h->P32[0].p, h->P32[1].p}, h->Xlo.p, h->U32.p, S->N32, S->M32, false, sizeof(zf)};
    }
    WorkSet *ws = &w64;
    bool lo = false;
    int since_flush = 0;

    int b = m1, bp = 0;
    int cur = 0, prev = 2, next = 1;
    int pcur = 0;  // P buffer holding P_{j,i-1}
    int status = DSBCG_OK;
    int iters = 0;
    const int steps = o.fixed_iters > 0 ? o.fixed_iters : o.max_iters;
    std::vector<int32_t> act;

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
    auto flush = [&](void) -> int {
        // X_hi += X_lo, X_lo = 0 (FP64 solution accumulation)
        PROF_LAUNCH(h, kProfConvert, copy_bytes(c.V, m * s, 8, 16, true), st,
                    copy_field(false, true, c.V, m * s, h->Xlo.p, m * s, kPlane, 0, h->X.p, m * s,
                               kPlane, true, 1.0, st));
        HIPCHK(hipMemsetAsync(h->Xlo.p, 0, (size_t)n * m * s * sizeof(zf), st));
        since_flush = 0;
        stt.reliable_updates += 1;
        return DSBCG_OK;
    };
    active_list();
    bool done = (m1 == 0) || (act.empty() && o.fixed_iters <= 0);

    for (int i = 1; !done && i <= steps; ++i) {
        if (form32 && !lo && max_active_est() <= switch_at) {
            // continue the same recurrences with FP32 vectors
            CHK(convert_block(h, c.V, b, w64.V[cur], true, w32.V[cur], false, st));
            if (i > 1) {
                CHK(convert_block(h, c.V, bp, w64.V[prev], true, w32.V[prev], false, st));
                for (int j : act)
                    CHK(convert_block(h, c.V, bp, (zd *)w64.P[pcur] + (int64_t)j * n * wmax, true,
                                      (zf *)w32.P[pcur] + (int64_t)j * n * wmax, false, st));
            }
            HIPCHK(hipMemsetAsync(h->Xlo.p, 0, (size_t)n * m * s * sizeof(zf), st));
            ws = &w32;
            lo = true;
            since_flush = 0;
            stt.switch_iter = i;
        }
        const bool f64 = ws->fp64;
        Ts ts{h, f64, st, n};
        iters = i;
        stt.mvms += b;
        void *Vc = ws->V[cur], *Vp = ws->V[prev], *Vn = ws->V[next];
        // W = A V_i
        CHK(apply_A_plane(h, f64, ws->U, kappa, Vc, ws->T, ws->W, b, st));
        // alpha_i = V_i^H (W - V_{i-1} beta_i^H)
        {
            TsArgs a = ts_args();
            a.K = (i > 1) ? 2 : 1;
            a.X[0] = ws->W; a.ldx[0] = b; a.bx[0] = b; a.C[0] = nullptr;
            a.X[1] = Vp; a.ldx[1] = bp; a.bx[1] = bp; a.C[1] = coef_slot(h, 0);
            a.bout = b;
            a.gram = 2; a.L = Vc; a.ldl = b; a.bl = b;
            CHK(ts.run_reduce(a, b, 0));
        }
        // hermitised alpha_i, -alpha_i as a coefficient
        PROF_LAUNCH(h, kProfSmall, 0.0, st, small_prep_alpha(S, red_slot(h, 0), st));
        // per-shift coefficients and P_j / X_j updates
        for (size_t q = 0; q < act.size(); ++q) h->list_host[q] = act[q];
        HIPCHK(hipMemcpyAsync(h->list.p, h->list_host, act.size() * sizeof(int32_t) + 4,
                              hipMemcpyHostToDevice, st));
        PROF_LAUNCH(h, kProfSmall, 0.0, st,
                    small_shift_coeffs(S, rep, red_slot(h, 0), i == 1, (const int32_t *)h->list.p,
                                       (int)act.size(), st));
        if (!act.empty()) {
            ShiftArgs sa;
            sa.nrows = n;
            sa.V = Vc;
            sa.b = b;
            sa.bp = bp;
            sa.m = m;
            sa.Pold = ws->P[pcur];
            sa.Pnew = ws->P[pcur ^ 1];
            sa.pstride = n * wmax;
            sa.X = ws->X;
            sa.xstride = n * m;
            sa.N = ws->N;
            sa.M = ws->M;
            sa.shifts = (const int32_t *)h->list.p;
            sa.nshift = (int)act.size();
            sa.colmask = rep->colmask;
            sa.first = (i == 1);
            PROF_LAUNCH(h, kProfShift, shift_bytes(sa, f64), st, shift_update(f64, sa, st));
        }
        // W <- W - V_i alpha_i - V_{i-1} beta_i^H  and  G1 = W^H W
        {
            TsArgs a = ts_args();
            a.K = (i > 1) ? 3 : 2;
            a.X[0] = ws->W; a.ldx[0] = b; a.bx[0] = b; a.C[0] = nullptr;
            a.X[1] = Vc; a.ldx[1] = b; a.bx[1] = b; a.C[1] = coef_slot(h, 1);
            a.X[2] = Vp; a.ldx[2] = bp; a.bx[2] = bp; a.C[2] = coef_slot(h, 0);
            a.bout = b;
            a.out = ws->W; a.ldo = b;
            a.gram = 1;
            CHK(ts.run_reduce(a, b, 1));
        }
        // first CholQR pass with deflation
        PROF_LAUNCH(h, kProfSmall, 0.0, st,
                    small_chol_deflate(S, rep, red_slot(h, 0), red_slot(h, 1),
                                       lo ? std::max(c.o.tau_W, 1e-8) : c.o.tau_W, st));
        // second pass: G2 = (W C1)^H (W C1); C1 has zero columns past the new width
        {
            TsArgs a = ts_args();
            a.K = 1;
            a.X[0] = ws->W; a.ldx[0] = b; a.bx[0] = b; a.C[0] = S->C1;
            a.bout = b;
            a.gram = 1;
            CHK(ts.run_reduce(a, b, 2));
        }
        PROF_LAUNCH(h, kProfSmall, 0.0, st,
                    small_finish(S, rep, red_slot(h, 2), tol, o.freeze, (const int32_t *)h->list.p,
                                 (int)act.size(), st));
        // V_{i+1} = W Rinv (width b, zero columns past the new width)
        {
            TsArgs a = ts_args();
            a.K = 1;
            a.X[0] = ws->W; a.ldx[0] = b; a.bx[0] = b; a.C[0] = S->Rinv;
            a.bout = b;
            a.out = Vn; a.ldo = b;
            CHK(ts.run(a, nullptr));
        }
        if (lo && ++since_flush >= std::max(1, o.ru_interval)) CHK(flush());
        CHK(read_report(h, st));
        const StepReport &R = *h->rep_host;
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
        if (bnew > 0 && bnew < b) {
            // compact V_{i+1} to leading dimension bnew, into the buffer of V_{i-1}
            PROF_LAUNCH(h, kProfConvert, copy_bytes(c.V, bnew, ws->esz, ws->esz, false), st,
                        copy_field(f64, f64, c.V, bnew, Vn, b, kPlane, 0, Vp, bnew, kPlane, false, 1.0, st));
            std::swap(prev, next);
        }
        active_list();
        if (bnew == 0) done = true;
        if (o.fixed_iters <= 0 && act.empty()) done = true;
        // rotate the three-block window
        const int old_prev = prev;
        prev = cur;
        cur = next;
        next = old_prev;
        pcur ^= 1;
        bp = b;
        b = bnew;
        stt.final_width = bnew;
    }
    if (lo) CHK(flush());
    stt.block_iters += iters;
    if (status == DSBCG_OK && !done && o.fixed_iters <= 0)
        status = fail(DSBCG_ERR_NOT_CONVERGED, "max_iters reached");
    // iterates to the caller's layout
    for (int j = 0; j < s; ++j)
        PROF_LAUNCH(h, kProfConvert, copy_bytes(c.V, m, 16, 16, false), st,
                    copy_field(true, true, c.V, m, (const zd *)h->X.p + (int64_t)j * n * m, m, kPlane, 0,
                               (zd *)Xapi + (int64_t)j * n * m, m, kApi, false, 1.0, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int j = 0; j < s; ++j)
        for (int l = 0; l < m; ++l) stt.est[j * m + l] = h->rep_host->est[j][l];
    return status;
}

}  // namespace

extern "C" {

int dsbcg_solve(dsbcg_handle h, const void *U, double kappa, const void *B, int32_t m,
                const double *sigma, int32_t s, double tol, const dsbcg_opts *opts, void *X,
                dsbcg_stats *stats, dsbcg_stream stream) {
    if (!h || !U || !B || !sigma || !X) return fail(DSBCG_ERR_ARG, "NULL argument");
    if (m < 1 || m > DSBCG_MAX_RHS) return fail(DSBCG_ERR_ARG, "m out of range");
    if (s < 1 || s > DSBCG_MAX_SHIFTS) return fail(DSBCG_ERR_ARG, "s out of range");
    if (!(tol > 0) || !std::isfinite(tol)) return fail(DSBCG_ERR_ARG, "tol must be > 0");
    if (!std::isfinite(kappa)) return fail(DSBCG_ERR_ARG, "kappa not finite");
    for (int j = 0; j < s; ++j)
        if (!std::isfinite(sigma[j])) return fail(DSBCG_ERR_ARG, "sigma not finite");
    dsbcg_opts o;
    dsbcg_default_opts(&o);
    if (opts) o = *opts;
    if (o.precision != DSBCG_FP64 && o.precision != DSBCG_FP32_RELIABLE)
        return fail(DSBCG_ERR_ARG, "unknown precision");
    if (o.tau_B < 0) o.tau_B = 0.1 * tol;
    if (o.tau_W < 0) o.tau_W = 1e-12;
    if (o.max_iters < 1) o.max_iters = 1;
    if (o.switch_at < 0) o.switch_at = std::min(1e-2, 1e6 * tol);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = 12 * (int64_t)h->g.V;

    SolveStats stt;
    int status = solve_core(h, U, kappa, B, m, sigma, s, tol, o, o.switch_at, X, stt, st);
    if (status != DSBCG_OK && status != DSBCG_ERR_NOT_CONVERGED) return status;

    // FP64 true residuals of every system; re-solve the shifts that miss tol
    std::vector<double> tr((size_t)s * m, 0.0);
    const bool want_true = (stats && stats->true_relres) || o.refine;
    if (want_true && status == DSBCG_OK) {
        CHK(true_residuals(h, st, U, kappa, B, X, m, sigma, s, tr.data(), -1, nullptr));
        for (int round = 0; o.refine && round < 2; ++round) {
            bool any = false;
            for (int j = 0; j < s; ++j) {
                double worst = 0.0;
                for (int l = 0; l < m; ++l) worst = std::max(worst, tr[j * m + l]);
                if (worst <= tol) continue;
                any = true;
                // residual block R_j, then (sigma_j + A) E = R_j in FP64 and X_j += E
                CHK(ensure(h->Rres, (size_t)n * m * sizeof(zd)));
                CHK(ensure(h->Xref, (size_t)n * m * sizeof(zd)));
                std::vector<double> tmp((size_t)s * m);
                CHK(true_residuals(h, st, U, kappa, B, X, m, sigma, s, tmp.data(), j, h->Rres.p));
                double ratio = 1e300;
                for (int l = 0; l < m; ++l)
                    if (tr[j * m + l] > 0) ratio = std::min(ratio, 1.0 / tr[j * m + l]);
                dsbcg_opts ro = o;
                ro.precision = DSBCG_FP64;
                ro.fixed_iters = 0;
                ro.tau_B = 0.1 * tol;
                SolveStats rs;
                const double rtol = std::max(0.5 * tol * ratio, 1e-15);
                int rc = solve_core(h, U, kappa, h->Rres.p, m, &sigma[j], 1, rtol, ro, 0.0, h->Xref.p, rs, st);
                if (rc != DSBCG_OK && rc != DSBCG_ERR_NOT_CONVERGED) return rc;
                stt.refine_iters += rs.block_iters;
                stt.mvms += rs.mvms;
                PROF_LAUNCH(h, kProfConvert, copy_bytes(h->g.V, m, 16, 16, true), st,
                            copy_field(true, true, h->g.V, m, h->Xref.p, m, kApi, 0,
                                       (zd *)X + (int64_t)j * n * m, m, kApi, true, 1.0, st));
            }
            if (!any) break;
            CHK(true_residuals(h, st, U, kappa, B, X, m, sigma, s, tr.data(), -1, nullptr));
        }
        double worst = 0.0;
        for (double v : tr) worst = std::max(worst, v);
        if (worst > tol && o.fixed_iters <= 0)
            status = fail(DSBCG_ERR_NOT_CONVERGED, "true relative residual " + std::to_string(worst) +
                                                       " above tol after refinement");
    }
    if (stats) {
        double *est = stats->est_relres, *tru = stats->true_relres;
        if (est) std::copy(stt.est, stt.est + (size_t)s * m, est);
        if (tru) std::copy(tr.begin(), tr.end(), tru);
        stats->block_iters = stt.block_iters;
        stats->rank0 = stt.rank0;
        stats->deflations = stt.deflations;
        stats->reliable_updates = stt.reliable_updates;
        stats->refine_iters = stt.refine_iters;
        stats->final_width = stt.final_width;
        stats->switch_iter = stt.switch_iter;
        stats->mvms = stt.mvms;
    }
    return status;
}

int dsbcg_link_grad(dsbcg_handle h, double kappa, const void *Phi, const void *Psi, int32_t nvec,
                    void *dU, dsbcg_stream stream) {
    (void)h; (void)kappa; (void)Phi; (void)Psi; (void)nvec; (void)dU; (void)stream;
    return fail(DSBCG_ERR_ARG, "link gradient not available in this build");
}

}  // extern "C"
