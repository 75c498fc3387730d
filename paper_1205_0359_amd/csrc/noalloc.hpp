// Internal interface of the entry point that allocates no device memory
// (noalloc.hip) with the rest of the library (solver.hip).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/dsbcg.h"
#include "stencil.hpp"

namespace dsbcg {

// Bytes of the per-device workspace of dsbcg_apply_A_noalloc.
constexpr size_t kNoallocScratchBytes = (size_t)128 << 20;

// Looks up, once per device, the address of that device's workspace (the
// device must be current).  Called by dsbcg_create.
int noalloc_setup(int device);

// Defined in solver.hip: the geometry, device and staged FP64 / FP32
// structure-of-arrays links (NULL when none are staged) of a handle, and the
// message of a failed call.
void handle_view(dsbcg_handle h, Geom *g, int *device, const void **ul64, const void **ul32);
int set_error(int code, const char *msg);

}  // namespace dsbcg
