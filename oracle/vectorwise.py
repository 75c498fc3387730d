"""Vector-wise stopping of DSBlockCG, FP64 -- TEST INFRASTRUCTURE ONLY.

The paper's iterates advance one Lanczos vector at a time (Sec. 3): the k-th
iterate is the Galerkin solution on the first k basis vectors,

    X^(k) = V^(k) (T_sigma^(k))^{-1} (V^(k))^H B                   (eq. (3.2))

with T_sigma^(k) = sigma I + T^(k) the leading k x k part of the banded
projected matrix, and its residual R^(k) = W^(k) C^(k) lies in the span of
the following basis vectors (the residual paragraph of Sec. 3), so that its
column norms are those of C^(k).  Stopping at this granularity lets each
system (l, j) stop at its own k instead of at the end of a block step.

This module states that definition plainly: the basis and T come from the
same block Lanczos steps as ``dsbcg.dsbcg`` (deflated QR of B, then
W = A V_i - V_{i-1} beta_i^H, alpha_i, W -= V_i alpha_i, deflated QR of W),
T is assembled densely from alpha_i and beta_{i+1}, and at every k the
k x k shifted system is solved densely:

    Y     = (T_sigma^(k))^{-1} (E rho)[1 : k]      (E rho = V^H B: B = V_1 rho)
    C^(k) = (E rho)[k+1 : k+w] - T[k+1 : k+w, 1 : k] Y
            (w: the rows of T known past k; the first term is nonzero only
            while k is below the rank of B, i.e. inside the first block)
    x_l   = V^(k) Y[:, l]  when ||C^(k)[:, l]|| <= tol ||b_l|| first holds.

No recurrence, blocking or update formula is used beyond that definition.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .dsbcg import _herm, deflated_qr


@dataclasses.dataclass
class VectorResult:
    X: np.ndarray                 # (s, n, m)
    iters: int = 0                # block steps taken
    mvms: int = 0                 # sum of the block widths (block-wise count)
    mvms_vector: int = 0          # the stage k at which the last system stopped
    rank0: int = 0
    widths: list = dataclasses.field(default_factory=list)
    est: np.ndarray | None = None           # (m, s) estimate at the stopping stage
    frozen_stage: np.ndarray | None = None  # (m, s) k at which (l, j) stopped (0: never)
    exhausted: bool = False


def stage_solution(T: np.ndarray, rho: np.ndarray, sigma: float, k: int, known: int):
    """Y = (sigma I + T[:k, :k])^{-1} (E rho)[:k] and C = (E rho)[k:known] - T[k:known, :k] Y.

    B - (sigma I + A) V^(k) Y = V ((E rho) - T_sigma[:, :k] Y), whose first k
    rows vanish by the choice of Y, so the residual is V[:, k:known] C.

    T: the dense projected matrix (at least known x known, entries past the
    computed band unused); rho: (r0, m) with r0 the rank of B; known: the
    number of rows of T whose first k columns are computed.
    """
    m = rho.shape[1]
    E = np.zeros((max(known, rho.shape[0]), m), dtype=np.complex128)
    E[:rho.shape[0]] = rho
    Ts = T[:k, :k] + sigma * np.eye(k)
    Y = np.linalg.solve(Ts, E[:k])
    C = E[k:known] - T[k:known, :k] @ Y
    return Y, C


def dsbcg_vectorwise(apply_A, B: np.ndarray, sigma, tol: float, max_iters: int = 10000,
                     tau_B: float | None = None, tau_W: float = 1e-12,
                     record: bool = False) -> VectorResult:
    """Solve (sigma_j I + A) X_j = B, each system stopping at its own stage k.

    The block steps and deflation rules are those of ``dsbcg.dsbcg``; after
    block step i the stages k = K_{i-1} + 1 .. K_i (K_i the number of basis
    vectors through block i) are examined in order, and system (l, j) stops
    at the first stage whose estimate ||C^(k)[:, l]|| / ||b_l|| is <= tol,
    with x_{l,j} = V^(k) Y[:, l].  Systems that never stop keep the iterate of
    the last stage reached.  With record=True the result also carries the
    basis (``Vall``) and T (``T``, ``known``) as attributes.
    """
    B = np.asarray(B, dtype=np.complex128)
    n, m = B.shape
    sigma = np.asarray(sigma, dtype=np.float64)
    s = len(sigma)
    if tau_B is None:
        tau_B = 0.1 * tol
    bnorm = np.linalg.norm(B, axis=0)
    safe = np.where(bnorm > 0, bnorm, 1.0)
    X = np.zeros((s, n, m), dtype=np.complex128)
    res = VectorResult(X=X)
    res.frozen_stage = np.zeros((m, s), dtype=np.int64)

    V1, rho, _ = deflated_qr(B, tau_B * bnorm)
    res.rank0 = V1.shape[1]
    est = np.zeros((m, s))
    for j in range(s):
        est[:, j] = np.linalg.norm(rho, axis=0) / safe
    res.est = est
    if V1.shape[1] == 0:
        res.exhausted = True
        return res
    active = np.ones((m, s), dtype=bool)
    active[bnorm == 0, :] = False

    blocks = [V1]
    T = np.zeros((0, 0), dtype=np.complex128)
    Vprev, beta = None, None
    Test = 0.0
    K_prev = 0
    last_Y = [None] * s
    for i in range(1, max_iters + 1):
        Vcur = blocks[-1]
        b = Vcur.shape[1]
        res.widths.append(b)
        res.mvms += b
        res.iters = i

        W = apply_A(Vcur)
        if Vprev is not None:
            W = W - Vprev @ beta.conj().T
        alpha = _herm(Vcur.conj().T @ W)
        W = W - Vcur @ alpha
        Test = max(Test, np.linalg.norm(alpha))
        if beta is not None:
            Test = max(Test, np.linalg.norm(beta))
        Vnext, beta_next, _ = deflated_qr(W, tau_W * Test)
        bn = Vnext.shape[1]

        # T through block i, with the rows of beta_{i+1} below it
        K_i = K_prev + b
        known = K_i + bn
        Tn = np.zeros((known, known), dtype=np.complex128)
        Tn[:T.shape[0], :T.shape[1]] = T[:known, :known]
        Tn[K_prev:K_i, K_prev:K_i] = alpha
        Tn[K_i:known, K_prev:K_i] = beta_next
        Tn[K_prev:K_i, K_i:known] = beta_next.conj().T
        T = Tn
        blocks.append(Vnext)
        Vall = np.concatenate(blocks, axis=1)

        for r in range(1, b + 1):
            k = K_prev + r
            for j in range(s):
                if not active[:, j].any():
                    continue
                Y, C = stage_solution(T, rho, sigma[j], k, known)
                e = np.linalg.norm(C, axis=0) / safe
                last_Y[j] = (k, Y)
                for l in range(m):
                    if not active[l, j]:
                        continue
                    est[l, j] = e[l]
                    if e[l] <= tol:
                        X[j][:, l] = Vall[:, :k] @ Y[:, l]
                        res.frozen_stage[l, j] = k
                        active[l, j] = False
        K_prev = K_i
        if bn == 0:
            res.exhausted = True
            break
        if not active.any():
            break
        Vprev, beta = Vcur, beta_next

    # systems that never stopped keep the iterate of the last stage
    for j in range(s):
        if last_Y[j] is None:
            continue
        k, Y = last_Y[j]
        for l in range(m):
            if active[l, j]:
                X[j][:, l] = Vall[:, :k] @ Y[:, l]
    res.est = est
    stopped = res.frozen_stage[bnorm > 0, :]
    res.mvms_vector = int(stopped.max()) if stopped.size and (stopped > 0).all() else K_prev
    if record:
        res.Vall, res.T, res.known = Vall, T, known
    return res
