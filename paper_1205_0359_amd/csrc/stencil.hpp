// Wilson-Dirac stencil launchers.
#pragma once

#include "common.hpp"

namespace dsbcg {

struct Geom {
    int32_t L[4];
    int32_t V;
};

// out = D in (dagger = false) or D^H in (dagger = true) on nb columns.
// Element (site x, spin-colour c, column r) of a field lives at
//   x * site_stride + c * comp_stride + r.
// fp64 selects double (U, in, out all double) or float data.
// lds_links stages each workgroup's link matrices in LDS.
hipError_t wilson_apply(const Geom &g, bool fp64, const void *U, double kappa, const void *in,
                        int64_t in_site, int64_t in_comp, void *out, int64_t out_site,
                        int64_t out_comp, int nb, bool dagger, bool lds_links, hipStream_t st);

// Neighbour table [V][8] (+x, -x, +y, -y, +z, -z, +t, -t) as the stencil computes it.
hipError_t neighbor_table(const Geom &g, int32_t *dev_out, hipStream_t st);

}  // namespace dsbcg
