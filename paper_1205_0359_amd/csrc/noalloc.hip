// dsbcg_apply_A_noalloc: Y = A X = D^H (D X) with no device allocation, for
// callers that cannot allocate (code under HIP graph capture, serving loops,
// harnesses that forbid it).  The column-major staging of X, the
// intermediate D X and (when the caller passes U) the structure-of-arrays
// links live in one workspace per device (the second pass writes Y in the
// caller's layout directly), a file-scope device array that
// each GPU the library runs on holds until the process ends.  The kernels
// are those of dsbcg_apply_A, launched in the same order, so the result is
// the same bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>

#include "blas.hpp"
#include "noalloc.hpp"

// The workspace.  In host code this name stands for the array but is not a
// device address: the kernels receive the address that hipGetSymbolAddress
// returns for the current device (g_scratch below).
static __device__ __align__(256) unsigned char scratch[dsbcg::kNoallocScratchBytes];

namespace dsbcg {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

int noalloc_setup(int device) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (device < 0 || device >= kMaxDevices) return set_error(DSBCG_ERR_HIP, "device index out of range");
    if (g_scratch[device]) return DSBCG_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        char msg[160];
        snprintf(msg, sizeof msg, "hipGetSymbolAddress of the no-allocation workspace: %s", hipGetErrorString(e));
        return set_error(DSBCG_ERR_HIP, msg);
    }
    g_scratch[device] = p;
    return DSBCG_OK;
}

}  // namespace dsbcg

using namespace dsbcg;

extern "C" int dsbcg_apply_A_noalloc(dsbcg_handle h, const void *U, double kappa, const void *X, void *Y,
                                     int32_t m, int32_t precision, dsbcg_stream stream) {
    if (!h || !X || !Y) return set_error(DSBCG_ERR_ARG, "NULL argument");
    if (m < 1 || m > DSBCG_MAX_RHS) return set_error(DSBCG_ERR_ARG, "m out of range");
    if (!std::isfinite(kappa)) return set_error(DSBCG_ERR_ARG, "kappa not finite");
    if (X == Y) return set_error(DSBCG_ERR_ARG, "Y must not alias X");
    if (precision != DSBCG_FP64 && precision != DSBCG_FP32_RELIABLE)
        return set_error(DSBCG_ERR_ARG, "unknown precision");
    const bool f64 = precision == DSBCG_FP64;
    Geom g;
    int device = -1;
    const void *ul64 = nullptr, *ul32 = nullptr;
    handle_view(h, &g, &device, &ul64, &ul32);
    const void *staged = f64 ? ul64 : ul32;
    if (!U && !staged) return set_error(DSBCG_ERR_ARG, "U is NULL and no links are staged on the handle");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device)
        return set_error(DSBCG_ERR_ARG, "the current device is not the handle's device");
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        base = (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
    }
    if (!base) return set_error(DSBCG_ERR_HIP, "the no-allocation workspace of this device is not set up");

    const int64_t V = g.V, n = 12 * V;
    const size_t esz = f64 ? 16 : 8;
    const size_t links_b = U ? round256((size_t)V * 36 * esz) : 0;
    const size_t block_b = round256((size_t)n * m * esz);
    const size_t need = links_b + 2 * block_b;
    if (need > kNoallocScratchBytes) {
        char msg[200];
        snprintf(msg, sizeof msg,
                 "dsbcg_apply_A_noalloc needs %zu bytes of workspace, the limit is %zu: use dsbcg_apply_A", need,
                 (size_t)kNoallocScratchBytes);
        return set_error(DSBCG_ERR_ARG, msg);
    }
    char *p = (char *)base;
    void *links = U ? (void *)p : const_cast<void *>(staged);
    void *xin = p + links_b, *tmp = p + links_b + block_b;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (U) e = links_to_soa(V, U, links, f64, st);
    if (e == hipSuccess)
        e = copy_field(V, m, FieldDesc{const_cast<void *>(X), kApi, m, 0, true}, FieldDesc{xin, kCM, n, 0, f64},
                       false, 1.0, st);
    const size_t colb = (size_t)n * esz;
    // D into tmp, then D^H of it straight into the caller's layout
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
        const char *in = (const char *)(pass ? tmp : xin);
        for (int c0 = 0; c0 < m && e == hipSuccess;) {
            const int k = stencil_chunk(f64, m - c0);
            const ApiOut ao{Y, m, c0};
            e = pass ? wilson_apply(g, f64, links, kappa, in + c0 * colb, nullptr, k, true, st, &ao)
                     : wilson_apply(g, f64, links, kappa, in + c0 * colb, (char *)tmp + c0 * colb, k, false, st);
            c0 += k;
        }
    }
    if (e != hipSuccess) {
        char msg[160];
        snprintf(msg, sizeof msg, "dsbcg_apply_A_noalloc: %s", hipGetErrorString(e));
        return set_error(DSBCG_ERR_HIP, msg);
    }
    return DSBCG_OK;
}
