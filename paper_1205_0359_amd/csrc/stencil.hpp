// Wilson-Dirac stencil launchers.
#pragma once

#include "common.hpp"

namespace dsbcg {

struct Geom {
    int32_t L[4];
    int32_t V;
};

// Output in the caller's layout: column r of a launch goes to column c0 + r
// of the complex128 field y [V][4][3][m] (site-major, column minor),
// widened from FP32 where the launch computes in FP32.
struct ApiOut {
    void *y;
    int32_t m, c0;
};

// out = D in (dagger = false) or D^H in (dagger = true) on nb <= 16 columns.
// in, out: column-major fields, element (column r, spin-colour c, site x) at
// (r*12 + c)*V + x.  Ul: links as structure of arrays, element e of U_mu(x)
// at (mu*9 + e)*V + x.  fp64 selects double or float data.  out must not
// alias in.  With api != nullptr the result goes to api->y instead of out
// (out unused).
hipError_t wilson_apply(const Geom &g, bool fp64, const void *Ul, double kappa, const void *in,
                        void *out, int nb, bool dagger, hipStream_t st, const ApiOut *api = nullptr);

// Columns of the first launch when a pass over nb columns is split into
// launches (the remainder is split by the same rule): FP64 passes over more
// than 7 columns run 5 columns at a time until at most 7 remain.
int stencil_chunk(bool fp64, int nb);

// True residual norms in one pass: with in = D x (column-major, nb columns,
// FP64), accumulates |b - sigma x - D^H in|^2 per column and workgroup into
// partials [nb][wilson_resid_workgroups(g)]; sum_columns adds them up in a
// fixed order into out[0..nb).
int wilson_resid_workgroups(const Geom &g);
hipError_t wilson_resid_norms(const Geom &g, const void *Ul, double kappa, const void *in, const void *b,
                              const void *x, double sigma, int nb, double *partials, hipStream_t st);
hipError_t sum_columns(const double *partials, int nwg, int nb, double *out, hipStream_t st);

// Links [V][4][3][3] (FP64) -> structure of arrays [4][9][V], FP64 or FP32.
hipError_t links_to_soa(int64_t V, const void *U, void *out, bool fp64, hipStream_t st);

// Neighbour table [V][8] (+x, -x, +y, -y, +z, -z, +t, -t) as the stencil computes it.
hipError_t neighbor_table(const Geom &g, int32_t *dev_out, hipStream_t st);

}  // namespace dsbcg
