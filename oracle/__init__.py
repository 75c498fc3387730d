"""CPU oracle for DSBlockCG -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It is a plain, slow FP64 statement of what the hot path
computes, written from the paper and sharing no code with the HIP library:

  * ``wilson_oracle.c``  the Wilson-Dirac operator D, D^H, A = D^H D, the
    neighbour table and the link derivative (C, loops over sites);
  * ``dsbcg.py``         the deflated shifted block CG method in block form
    (numpy), following Sec. 3 of the paper;
  * ``vectorwise.py``    the same method stopping each system at its own
    Lanczos vector, from the dense definition of the k-th iterate (eq. (3.2)).

Every function is pinned by CPU tests against facts fixed outside the oracle
(closed forms, textbook special cases, dense solves).
"""
from .wilson import (apply_D, apply_A, apply_D_sites, apply_A_sites, neighbors, gamma,
                     link_grad, max_threads, load)
from .dsbcg import (dsbcg, deflated_qr, true_relres, partial_fraction, NotHPD, Result)

__all__ = ["apply_D", "apply_A", "apply_D_sites", "apply_A_sites", "neighbors", "gamma",
           "link_grad", "max_threads", "load", "dsbcg", "deflated_qr", "true_relres",
           "partial_fraction", "NotHPD", "Result"]
from .grad import adjoint_gradients  # noqa: E402
from .vectorwise import dsbcg_vectorwise, stage_solution, VectorResult  # noqa: E402

__all__ += ["adjoint_gradients", "dsbcg_vectorwise", "stage_solution", "VectorResult"]
