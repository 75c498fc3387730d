"""Pins of the oracle's Wilson-Dirac operator against facts fixed outside it.

Checked: Clifford algebra of the gamma table, the neighbour table against
modular arithmetic, the free-field (unit link) plane-wave action and the dense
spectrum of A in closed form, gamma5-hermiticity, the adjoint identity for
D^H, hermiticity and positivity of A, gauge covariance (which fixes the
forward/backward link conventions), site-sampled evaluation and the link
derivative against finite differences.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1205_0359_amd import inputs


def _inner(a, b):
    return np.vdot(a.ravel(), b.ravel())


def _coords(L):
    V = int(np.prod(L))
    idx = np.arange(V)
    x = idx % L[0]
    y = (idx // L[0]) % L[1]
    z = (idx // (L[0] * L[1])) % L[2]
    t = idx // (L[0] * L[1] * L[2])
    return np.stack([x, y, z, t], axis=1)


def _site(L, c):
    return c[..., 0] + L[0] * (c[..., 1] + L[1] * (c[..., 2] + L[2] * c[..., 3]))


def _hop(L, mu, d):
    c = _coords(L)
    c[:, mu] = (c[:, mu] + d) % L[mu]
    return _site(L, c)


def _gammas():
    return [oracle.gamma(mu) for mu in range(4)]


def test_gamma_clifford_and_chirality():
    g = _gammas()
    for mu, nu in itertools.product(range(4), repeat=2):
        anti = g[mu] @ g[nu] + g[nu] @ g[mu]
        assert np.allclose(anti, 2.0 * (mu == nu) * np.eye(4), atol=0)
    for mu in range(4):
        assert np.array_equal(g[mu], g[mu].conj().T)
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    # chiral basis: gamma5 diagonal
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("L", [(3, 4, 5, 6), (4, 4, 4, 4), (2, 2, 2, 2)])
def test_neighbour_table_closed_form(L):
    nb = oracle.neighbors(L)
    for mu in range(4):
        assert np.array_equal(nb[:, 2 * mu], _hop(L, mu, +1))
        assert np.array_equal(nb[:, 2 * mu + 1], _hop(L, mu, -1))


def _Dp(p, kappa):
    """Free-field symbol: D(p) = 1 - 2 kappa sum cos p + 2 i kappa sum gamma sin p."""
    g = _gammas()
    out = (1 - 2 * kappa * np.sum(np.cos(p))) * np.eye(4, dtype=complex)
    for mu in range(4):
        out = out + 2j * kappa * np.sin(p[mu]) * g[mu]
    return out


def test_free_field_plane_wave():
    L = (4, 4, 4, 6)
    kappa = 0.12
    U = inputs.unit_links(L)
    rng = np.random.default_rng(11)
    c = _coords(L)
    for _ in range(3):
        nvec = rng.integers(0, 6, size=4) % np.array(L)
        p = 2 * np.pi * nvec / np.array(L)
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (c @ p))
        psi = phase[:, None, None] * chi[None]
        out = oracle.apply_D(L, U, kappa, psi)
        want = phase[:, None, None] * (_Dp(p, kappa) @ chi)[None]
        assert np.abs(out - want).max() < 1e-14
        outd = oracle.apply_D(L, U, kappa, psi, dagger=True)
        wantd = phase[:, None, None] * (_Dp(p, kappa).conj().T @ chi)[None]
        assert np.abs(outd - wantd).max() < 1e-14


def _dense(L, U, kappa, fn):
    V = int(np.prod(L))
    n = 12 * V
    E = np.eye(n, dtype=complex).reshape(n, V, 4, 3).transpose(1, 2, 3, 0)
    return fn(L, U, kappa, np.ascontiguousarray(E)).reshape(n, n)


@pytest.mark.slow
def test_free_field_spectrum_dense_4x4x4x4():
    # eigenvalues of A at unit links: a^2 + |b|^2, multiplicity 12 per momentum,
    # a = 1 - 2 kappa sum cos p, |b|^2 = 4 kappa^2 sum sin^2 p.
    L = (4, 4, 4, 4)
    kappa = 0.12
    A = _dense(L, inputs.unit_links(L), kappa, oracle.apply_A)
    w = np.linalg.eigvalsh(A)
    ks = 2 * np.pi * np.arange(4) / 4
    want = []
    for p in itertools.product(ks, repeat=4):
        p = np.array(p)
        a = 1 - 2 * kappa * np.cos(p).sum()
        want += [a * a + 4 * kappa ** 2 * (np.sin(p) ** 2).sum()] * 12
    want = np.sort(want)
    assert np.abs(w - want).max() < 1e-12
    assert abs(w[0] - (1 - 8 * kappa) ** 2) < 1e-13
    assert abs(w[-1] - (1 + 8 * kappa) ** 2) < 1e-12


@pytest.fixture(scope="module")
def haar_small():
    L = (4, 4, 2, 6)
    U = inputs.make_links(L, "haar", inputs.rng_for(900, 0))
    V = int(np.prod(L))
    rng = inputs.rng_for(900, 1)
    phi = inputs.complex_gaussian(rng, (V, 4, 3, 3))
    psi = inputs.complex_gaussian(rng, (V, 4, 3, 3))
    return L, U, phi, psi


def test_adjoint_identity(haar_small):
    L, U, phi, psi = haar_small
    k = 0.13
    lhs = _inner(phi, oracle.apply_D(L, U, k, psi))
    rhs = _inner(oracle.apply_D(L, U, k, phi, dagger=True), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-12


def test_gamma5_hermiticity(haar_small):
    L, U, phi, psi = haar_small
    k = 0.13
    g = _gammas()
    g5 = g[0] @ g[1] @ g[2] @ g[3]

    def G5(f):
        return np.einsum("ab,vbcm->vacm", g5, f)

    lhs = _inner(phi, oracle.apply_D(L, U, k, psi))
    rhs = _inner(G5(oracle.apply_D(L, U, k, G5(phi))), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # and therefore D^H = g5 D g5 as operators
    assert np.abs(oracle.apply_D(L, U, k, psi, dagger=True) - G5(oracle.apply_D(L, U, k, G5(psi)))).max() < 1e-13


def test_A_hermitian_positive(haar_small):
    L, U, phi, psi = haar_small
    k = 0.12
    Apsi = oracle.apply_A(L, U, k, psi)
    Aphi = oracle.apply_A(L, U, k, phi)
    assert abs(_inner(phi, Apsi) - np.conj(_inner(psi, Aphi))) < 1e-12 * abs(_inner(phi, Apsi))
    Dpsi = oracle.apply_D(L, U, k, psi)
    for r in range(psi.shape[3]):
        q = _inner(psi[..., r], Apsi[..., r])
        assert abs(q.imag) < 1e-12 * abs(q)
        assert abs(q.real - np.linalg.norm(Dpsi[..., r]) ** 2) < 1e-12 * q.real
        assert q.real > 0


def test_gauge_covariance(haar_small):
    L, U, phi, psi = haar_small
    k = 0.12
    V = int(np.prod(L))
    Om = inputs.haar_su3(inputs.rng_for(901, 0), V)
    UO = np.empty_like(U)
    for mu in range(4):
        fwd = _hop(L, mu, +1)
        UO[:, mu] = Om @ U[:, mu] @ np.conj(np.swapaxes(Om[fwd], -1, -2))

    def rot(f):
        return np.einsum("vab,vsbm->vsam", Om, f)

    for dag in (False, True):
        lhs = oracle.apply_D(L, UO, k, rot(psi), dagger=dag)
        rhs = rot(oracle.apply_D(L, U, k, psi, dagger=dag))
        assert np.abs(lhs - rhs).max() < 1e-13


def test_columns_independent(haar_small):
    L, U, phi, psi = haar_small
    k = 0.12
    full = oracle.apply_A(L, U, k, psi)
    for r in range(psi.shape[3]):
        one = oracle.apply_A(L, U, k, np.ascontiguousarray(psi[..., r]))
        assert np.array_equal(one, full[..., r])


def test_site_sampled_evaluation(haar_small):
    L, U, phi, psi = haar_small
    k = 0.12
    sites = np.array([0, 1, 17, 95, 191, 150])
    assert np.array_equal(oracle.apply_D_sites(L, U, k, psi, sites), oracle.apply_D(L, U, k, psi)[sites])
    assert np.array_equal(oracle.apply_D_sites(L, U, k, psi, sites, dagger=True),
                          oracle.apply_D(L, U, k, psi, dagger=True)[sites])
    full = oracle.apply_A(L, U, k, psi)[sites]
    assert np.abs(oracle.apply_A_sites(L, U, k, psi, sites) - full).max() < 1e-13


def test_link_derivative_finite_difference(haar_small):
    # f(U) = Re <phi, D[U] psi> is real-linear in U, so a central difference is
    # exact up to rounding: df = Re <G, dU> with G = df/dRe U + i df/dIm U.
    L, U, phi, psi = haar_small
    k = 0.12
    G = oracle.link_grad(L, k, phi, psi)
    rng = np.random.default_rng(5)
    for _ in range(3):
        dU = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
        h = 1e-3
        fp = _inner(phi, oracle.apply_D(L, U + h * dU, k, psi)).real
        fm = _inner(phi, oracle.apply_D(L, U - h * dU, k, psi)).real
        fd = (fp - fm) / (2 * h)
        an = np.vdot(G.ravel(), dU.ravel()).real
        assert abs(fd - an) < 1e-9 * abs(an)
    # one entry at a time, real and imaginary directions
    for (x, mu, a, b) in [(0, 0, 0, 0), (37, 3, 2, 1), (191, 1, 1, 2)]:
        for unit in (1.0, 1j):
            dU = np.zeros_like(U)
            dU[x, mu, a, b] = unit
            fp = _inner(phi, oracle.apply_D(L, U + dU, k, psi)).real
            fm = _inner(phi, oracle.apply_D(L, U - dU, k, psi)).real
            want = (fp - fm) / 2
            got = G[x, mu, a, b].real if unit == 1.0 else G[x, mu, a, b].imag
            assert abs(got - want) < 1e-11
