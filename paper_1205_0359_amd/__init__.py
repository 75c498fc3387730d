"""MI355X-native deflated shifted block CG (DSBlockCG) for Wilson fermions.

Solves (sigma_j I + A) X_j = B, A = D^H D, for m right-hand sides and s real
shifts at once (Birk & Frommer, Sec. 1 and Sec. 3).  The computation runs in
the HIP library libdsbcg.so (C ABI: include/dsbcg.h); this package holds the
ctypes binding, the seeded input generators and the build script.
"""
from ._lib import (DSBCG_FP32_RELIABLE, DSBCG_FP64, DSBCGError, Handle, NotConvergedError,
                   NotHPDError, dsbcg_apply_A, dsbcg_apply_A_noalloc, dsbcg_apply_D, dsbcg_link_grad, dsbcg_neighbors,
                   dsbcg_profile_enable, dsbcg_profile_read, dsbcg_profile_select, dsbcg_solve,
                   dsbcg_solve_multi,
                   dsbcg_solve_rational, dsbcg_grad, dsbcg_stage_links, dsbcg_release_workspace, default_opts, load)

__all__ = ["DSBCG_FP32_RELIABLE", "DSBCG_FP64", "DSBCGError", "Handle", "NotConvergedError",
           "NotHPDError", "dsbcg_apply_A", "dsbcg_apply_A_noalloc", "dsbcg_apply_D", "dsbcg_link_grad", "dsbcg_neighbors",
           "dsbcg_profile_enable", "dsbcg_profile_read", "dsbcg_profile_select", "dsbcg_solve",
           "dsbcg_solve_multi",
           "dsbcg_solve_rational", "dsbcg_grad", "dsbcg_stage_links", "dsbcg_release_workspace", "default_opts", "load"]
