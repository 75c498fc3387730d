"""Pins of the oracle's adjoint gradients.

For L = sum_j alpha_j Re tr(B^H X_j) the B and sigma derivatives have closed
forms (dL/dB = 2 sum_j alpha_j X_j, half of it through X_j;
dL/dsigma_j = -alpha_j ||X_j||_F^2); the
link derivative is checked by central finite differences of L on a 2^4 lattice
with dense solves (the map is real-analytic in Re U and Im U)."""
import numpy as np

import oracle
from paper_1205_0359_amd import inputs


def _dense_A(L, U, kappa):
    V = int(np.prod(L))
    n = 12 * V
    E = np.eye(n, dtype=complex).reshape(n, V, 4, 3).transpose(1, 2, 3, 0)
    return oracle.apply_A(L, U, kappa, np.ascontiguousarray(E)).reshape(n, n)


def _loss(L, U, kappa, B, sigma, alpha):
    V = int(np.prod(L))
    n = 12 * V
    A = _dense_A(L, U, kappa)
    Bm = B.reshape(n, -1)
    tot = 0.0
    for j, sg in enumerate(sigma):
        X = np.linalg.solve(A + sg * np.eye(n), Bm)
        tot += alpha[j] * np.vdot(Bm.ravel(), X.ravel()).real
    return tot


def _setup(L, seed, m=2, s=3):
    V = int(np.prod(L))
    U = inputs.make_links(L, "haar", inputs.rng_for(seed, 0))
    B = inputs.gaussian_rhs(inputs.rng_for(seed, 1), V, m)
    sigma = np.logspace(-3, 0, s)
    alpha = inputs.rng_for(seed, 2).uniform(0.1, 1.0, s)
    return U, B, sigma, alpha


def _solve_all(L, U, kappa, B, sigma):
    V = int(np.prod(L))
    n = 12 * V
    A = _dense_A(L, U, kappa)
    return np.stack([np.linalg.solve(A + sg * np.eye(n), B.reshape(n, -1)).reshape(B.shape)
                     for sg in sigma])


def test_closed_forms_for_trace_loss():
    L = (2, 2, 2, 4)
    kappa = 0.12
    U, B, sigma, alpha = _setup(L, 950)
    X = _solve_all(L, U, kappa, B, sigma)
    G = np.stack([alpha[j] * B for j in range(len(sigma))])
    dU, dB, dsig, Lam = oracle.adjoint_gradients(L, U, kappa, B, sigma, X, G, tol=1e-13)
    # the path through X_j carries half of d/dB of sum_j alpha_j Re <B, X_j>; the
    # explicit B in the loss carries the other half (total 2 sum_j alpha_j X_j)
    want_B = sum(alpha[j] * X[j] for j in range(len(sigma)))
    assert np.abs(dB - want_B).max() < 1e-9 * np.abs(want_B).max()
    want_s = np.array([-alpha[j] * np.linalg.norm(X[j]) ** 2 for j in range(len(sigma))])
    assert np.allclose(dsig, want_s, rtol=1e-9)
    # Lambda_j = alpha_j X_j for this loss
    for j in range(len(sigma)):
        assert np.abs(Lam[j] - alpha[j] * X[j]).max() < 1e-9 * np.abs(X[j]).max()


def test_link_derivative_against_finite_differences():
    L = (2, 2, 2, 4)
    kappa = 0.12
    U, B, sigma, alpha = _setup(L, 951)
    X = _solve_all(L, U, kappa, B, sigma)
    G = np.stack([alpha[j] * B for j in range(len(sigma))])
    dU, _, _, _ = oracle.adjoint_gradients(L, U, kappa, B, sigma, X, G, tol=1e-13)
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(6):
        x, mu, a, b = rng.integers(0, 32), rng.integers(0, 4), rng.integers(0, 3), rng.integers(0, 3)
        for unit in (1.0, 1j):
            Up = U.copy()
            Up[x, mu, a, b] += h * unit
            Um = U.copy()
            Um[x, mu, a, b] -= h * unit
            fd = (_loss(L, Up, kappa, B, sigma, alpha) - _loss(L, Um, kappa, B, sigma, alpha)) / (2 * h)
            an = dU[x, mu, a, b].real if unit == 1.0 else dU[x, mu, a, b].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (x, mu, a, b, unit, fd, an)


def test_sigma_and_B_against_finite_differences():
    L = (2, 2, 2, 4)
    kappa = 0.12
    U, B, sigma, alpha = _setup(L, 952)
    X = _solve_all(L, U, kappa, B, sigma)
    # a general upstream gradient (not proportional to B)
    G = inputs.complex_gaussian(inputs.rng_for(952, 3), X.shape)
    _, dB, dsig, _ = oracle.adjoint_gradients(L, U, kappa, B, sigma, X, G, tol=1e-13)

    def loss(Bv, sv):
        Xv = _solve_all(L, U, kappa, Bv, sv)
        return sum(np.vdot(G[j].ravel(), Xv[j].ravel()).real for j in range(len(sv)))

    h = 1e-6
    for j in range(len(sigma)):
        sp, sm = sigma.copy(), sigma.copy()
        sp[j] += h
        sm[j] -= h
        fd = (loss(B, sp) - loss(B, sm)) / (2 * h)
        assert abs(fd - dsig[j]) <= 1e-6 * max(1.0, abs(dsig[j]))
    idx = (5, 1, 2, 0)
    for unit in (1.0, 1j):
        Bp, Bm_ = B.copy(), B.copy()
        Bp[idx] += h * unit
        Bm_[idx] -= h * unit
        fd = (loss(Bp, sigma) - loss(Bm_, sigma)) / (2 * h)
        an = dB[idx].real if unit == 1.0 else dB[idx].imag
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
