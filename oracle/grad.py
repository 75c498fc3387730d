"""Gradients of losses of the solutions X_j -- TEST INFRASTRUCTURE ONLY.

The paper does not differentiate its solver; this is the adjoint method for
X_j = (sigma_j I + A)^{-1} B with A = D^H D hermitian:

  dL = sum_j Re <G_j, dX_j>,  G_j = dL/dRe X_j + i dL/dIm X_j
  dX_j = (sigma_j + A)^{-1} (dB - dsigma_j X_j - dA X_j)
  Lambda_j = (sigma_j + A)^{-1} G_j
  dL/dB = sum_j Lambda_j,   dL/dsigma_j = -Re <Lambda_j, X_j>,
  dL/dU = -sum_j [ d/dU Re <D X_j, dD Lambda_j> + d/dU Re <D Lambda_j, dD X_j> ]

with dA = dD^H D + D^H dD.  Solves use the oracle's DSBlockCG; the link
derivative uses the oracle's link_grad (pinned by finite differences).
"""
from __future__ import annotations

import numpy as np

from .dsbcg import dsbcg
from .wilson import apply_A, apply_D, link_grad


def adjoint_gradients(L, U, kappa, B, sigma, X, G, tol=1e-12):
    """dL/dU (V,4,3,3), dL/dB (V,4,3,m), dL/dsigma (s,) for upstream G_j.

    B: (V,4,3,m); X, G: (s,V,4,3,m).
    """
    V = int(np.prod(L))
    n = 12 * V
    m = B.shape[-1]
    s = len(sigma)

    def op(Y):
        return apply_A(L, U, kappa, np.ascontiguousarray(Y).reshape(V, 4, 3, -1)).reshape(n, -1)

    Lam = np.zeros_like(X)
    for j in range(s):
        r = dsbcg(op, G[j].reshape(n, m), [sigma[j]], tol)
        Lam[j] = r.X[0].reshape(V, 4, 3, m)
    dB = Lam.sum(axis=0)
    dsig = np.array([-np.vdot(Lam[j].ravel(), X[j].ravel()).real for j in range(s)])
    dU = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    for j in range(s):
        DX = apply_D(L, U, kappa, X[j])
        DLam = apply_D(L, U, kappa, Lam[j])
        dU -= link_grad(L, kappa, DX, Lam[j])
        dU -= link_grad(L, kappa, DLam, X[j])
    return dU, dB, dsig, Lam
