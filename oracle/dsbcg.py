"""Deflated shifted block CG in block form, FP64 -- TEST INFRASTRUCTURE ONLY.

Plain numpy statement of the method of Sec. 3 of the paper, for the systems
(sigma_j I + A) X_j = B, j = 1..s (Sec. 1, eqs. (1.1), (1.2)).  The paper
gives no listing; this block form is the reading used throughout:

  Step 0  deflated QR of B in column order (drop a column whose remainder,
          after classical Gram-Schmidt applied twice, is at most
          tau_B * ||b_l||): B = V_1 rho.  Deflation = removing vectors that
          became linearly dependent (Sec. 1; Sec. 3 after eq. (3.1)).
  Step i  block Lanczos (Sec. 3, eq. (3.1): T = V^H A V hermitian and banded):
            W = A V_i - V_{i-1} beta_i^H
            alpha_i = herm(V_i^H W);  W <- W - V_i alpha_i
            W = V_{i+1} beta_{i+1}   (deflated QR, absolute threshold
                                      tau_W * ||T||_est)
          per shift, the block root-free Cholesky (L D L^H) of
          T_sigma = sigma I + T (Sec. 3, the update after eq. (3.2) and the
          shifted paragraph):
            Delta_{j,1} = alpha_1 + sigma_j I,   P_{j,1} = V_1,   Z_{j,1} = rho
            N_{j,i}     = Delta_{j,i-1}^{-1} beta_i^H
            Delta_{j,i} = alpha_i + sigma_j I - beta_i N_{j,i}
            P_{j,i}     = V_i - P_{j,i-1} N_{j,i}
            M_{j,i}     = Delta_{j,i}^{-1} Z_{j,i}
            X_j[:, l]  += P_{j,i} M_{j,i}[:, l]   for the unconverged l
            C_j         = -beta_{i+1} M_{j,i} = Z_{j,i+1}
          the residual is R_j = V_{i+1} C_j, so its column norms are those of
          C_j (Sec. 3, the residual paragraph); a system (l, j) stops being
          updated once ||C_j[:, l]|| <= tol ||b_l|| (Sec. 4).

The deflated QR here is classical Gram-Schmidt applied twice, column by
column; any QR with a positive real R diagonal gives the same factors in
exact arithmetic.
"""
from __future__ import annotations

import dataclasses

import numpy as np


class NotHPD(ArithmeticError):
    """A shifted block Delta_{j,i} is not positive definite: sigma_j I + A is not hpd."""


@dataclasses.dataclass
class Result:
    X: np.ndarray                 # (s, n, m)
    iters: int = 0                # block steps taken
    mvms: int = 0                 # applications of A to one vector: sum of block widths
    rank0: int = 0                # width of V_1 after deflating B
    widths: list = dataclasses.field(default_factory=list)   # m_i per step
    est: np.ndarray | None = None  # (m, s) last estimated relative residuals
    history: list = dataclasses.field(default_factory=list)  # est per step
    frozen_at: np.ndarray | None = None  # (m, s) step at which (l, j) stopped updating
    Vs: list | None = None        # recorded Lanczos blocks V_1, V_2, ...
    alphas: list | None = None
    betas: list | None = None     # beta_2, beta_3, ... (beta_{i+1} is m_{i+1} x m_i)
    rho: np.ndarray | None = None
    exhausted: bool = False       # the block Krylov space became invariant


def _herm(M: np.ndarray) -> np.ndarray:
    return 0.5 * (M + M.conj().T)


def deflated_qr(W: np.ndarray, thresh) -> tuple[np.ndarray, np.ndarray, list]:
    """Column-ordered QR with deflation.

    W (n x k); thresh is a scalar or per-column array.  Column l is orthogonalised
    against the vectors kept so far by classical Gram-Schmidt applied twice; it is
    kept (normalised) if the remainder norm exceeds thresh[l], else dropped.
    Returns Q (n x r), R (r x k) with W ~= Q R and the kept column indices.
    """
    n, k = W.shape
    thresh = np.broadcast_to(np.asarray(thresh, dtype=np.float64), (k,))
    cols = []
    coef = []          # coef[l] = projection coefficients of column l on the kept vectors
    kept = []
    for l in range(k):
        w = W[:, l].astype(np.complex128, copy=True)
        c = np.zeros(len(cols), dtype=np.complex128)
        for _ in range(2):
            if cols:
                Q = np.stack(cols, axis=1)
                d = Q.conj().T @ w
                w = w - Q @ d
                c = c + d
        nu = np.linalg.norm(w)
        if nu > thresh[l]:
            cols.append(w / nu)
            c = np.append(c, nu)
            kept.append(l)
        coef.append(c)
    r = len(cols)
    Q = np.stack(cols, axis=1) if cols else np.zeros((n, 0), dtype=np.complex128)
    R = np.zeros((r, k), dtype=np.complex128)
    for l, c in enumerate(coef):
        R[:len(c), l] = c
    return Q, R, kept


def _chol_solve(Lc: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Solve (Lc Lc^H) X = Y with the lower Cholesky factor Lc."""
    import scipy.linalg as sla
    Z = sla.solve_triangular(Lc, Y, lower=True)
    return sla.solve_triangular(Lc.conj().T, Z, lower=False)


def dsbcg(apply_A, B: np.ndarray, sigma, tol: float, max_iters: int = 10000,
          fixed_iters: int = 0, tau_B: float | None = None, tau_W: float = 1e-12,
          record: bool = False, freeze: bool = True) -> Result:
    """Solve (sigma_j I + A) X_j = B for all shifts.

    apply_A: callable mapping an (n, b) complex array to A times it.
    B: (n, m).  sigma: real shifts.  Stops when every (l, j) has an estimated
    relative residual <= tol, when the block Krylov space is exhausted, or
    after max_iters steps; with fixed_iters > 0 it runs exactly that many
    steps (unless exhausted earlier).  X^(0) = 0.
    """
    B = np.asarray(B, dtype=np.complex128)
    n, m = B.shape
    sigma = np.asarray(sigma, dtype=np.float64)
    s = len(sigma)
    if tau_B is None:
        tau_B = 0.1 * tol
    bnorm = np.linalg.norm(B, axis=0)
    X = np.zeros((s, n, m), dtype=np.complex128)
    res = Result(X=X)
    res.frozen_at = np.full((m, s), -1, dtype=np.int64)

    # Step 0: deflated QR of B.
    V1, rho, _ = deflated_qr(B, tau_B * bnorm)
    res.rank0 = V1.shape[1]
    res.rho = rho
    est = np.zeros((m, s))
    safe = np.where(bnorm > 0, bnorm, 1.0)
    for j in range(s):
        est[:, j] = np.linalg.norm(rho, axis=0) / safe
    res.est = est.copy()
    if record:
        res.Vs, res.alphas, res.betas = [V1.copy()], [], []
    if V1.shape[1] == 0:
        res.exhausted = True
        return res

    active = np.ones((m, s), dtype=bool)
    active[bnorm == 0, :] = False
    shift_on = active.any(axis=0)

    Vprev = None
    Vcur = V1
    beta = None                      # beta_i  (m_i x m_{i-1})
    Z = [rho.copy() for _ in range(s)]
    P = [None] * s
    Lprev = [None] * s               # Cholesky factor of Delta_{j,i-1}
    Test = 0.0
    steps = fixed_iters if fixed_iters > 0 else max_iters

    for i in range(1, steps + 1):
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

        M = [None] * s
        for j in range(s):
            if not shift_on[j]:
                continue
            if i == 1:
                Delta = alpha + sigma[j] * np.eye(b)
                P[j] = Vcur.copy()
            else:
                N = _chol_solve(Lprev[j], beta.conj().T)
                Delta = _herm(alpha + sigma[j] * np.eye(b) - beta @ N)
                P[j] = Vcur - P[j] @ N
            try:
                Lc = np.linalg.cholesky(Delta)
            except np.linalg.LinAlgError as e:
                raise NotHPD(f"Delta for shift {j} at step {i} is not positive definite") from e
            Lprev[j] = Lc
            M[j] = _chol_solve(Lc, Z[j])
            act = active[:, j]
            X[j][:, act] += P[j] @ M[j][:, act]

        Vnext, beta_next, _ = deflated_qr(W, tau_W * Test)
        if record:
            res.alphas.append(alpha.copy())
            res.betas.append(beta_next.copy())
            res.Vs.append(Vnext.copy())

        for j in range(s):
            if not shift_on[j]:
                continue
            C = -beta_next @ M[j]
            Z[j] = C
            est[:, j] = np.linalg.norm(C, axis=0) / safe
        res.est = est.copy()
        res.history.append(est.copy())

        if freeze:
            newly = active & (est <= tol)
            res.frozen_at[newly] = i
            active &= ~newly
            shift_on = active.any(axis=0)

        if Vnext.shape[1] == 0:
            res.exhausted = True
            break
        if fixed_iters <= 0 and not active.any():
            break

        Vprev, Vcur, beta = Vcur, Vnext, beta_next

    return res


def true_relres(apply_A, B: np.ndarray, sigma, X: np.ndarray) -> np.ndarray:
    """||b_l - (sigma_j + A) x_{l,j}|| / ||b_l||, shape (m, s) (Sec. 4: relative residual)."""
    B = np.asarray(B)
    s = len(sigma)
    m = B.shape[1]
    out = np.zeros((m, s))
    bnorm = np.linalg.norm(B, axis=0)
    safe = np.where(bnorm > 0, bnorm, 1.0)
    for j in range(s):
        R = B - sigma[j] * X[j] - apply_A(X[j])
        out[:, j] = np.linalg.norm(R, axis=0) / safe
    return out


def partial_fraction(B: np.ndarray, X: np.ndarray, coef, c0: float) -> np.ndarray:
    """Y = c0 B + sum_j coef_j X_j with X_j = (sigma_j I + A)^{-1} B.

    The partial-fraction form of a rational function of A applied to B (Sec. 1:
    the rational approximation that the rational hybrid Monte Carlo algorithm
    uses for a power of A, written as a partial fraction expansion, is the
    source of the shifted systems).  B: (n, m); X: (s, n, m).
    """
    Y = c0 * np.asarray(B, dtype=np.complex128)
    for j, c in enumerate(coef):
        Y = Y + c * X[j]
    return Y

