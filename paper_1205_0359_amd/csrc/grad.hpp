// Link derivative of sum_k Re <Phi_k, D[U] Psi_k>.
#pragma once

#include "common.hpp"
#include "stencil.hpp"

namespace dsbcg {

// dU (=|+=) scale * d/dU of sum_k Re <Phi_k, D Psi_k> over cols column-major
// columns of Phi and Psi (FP64), in the convention dRe + i dIm; dU is
// [V][4][3][3].
hipError_t link_grad_apply(const Geom &g, double kappa, const void *Phi, const void *Psi, int cols,
                           void *dU, bool accumulate, double scale, hipStream_t st);

}  // namespace dsbcg
