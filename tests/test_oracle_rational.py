"""Pins of the oracle's partial-fraction form Y = c0 B + sum_j c_j (sigma_j + A)^{-1} B.

Checked against facts fixed outside the oracle: the scalar rational function
on a diagonal operator (each component of Y is r(d_i) b_i with
r(x) = c0 + sum_j c_j / (sigma_j + x)); the product identity
1 / ((x + s1)(x + s2)) = [1/(x + s1) - 1/(x + s2)] / (s2 - s1), checked by
applying (s2 + A)(s1 + A) to Y with the Wilson operator (matrix-vector
products only); and the limits c = 0 (Y = c0 B) and one shift with c0 = 0
(Y = X_1).
"""
import numpy as np
import pytest

import oracle
from paper_1205_0359_amd import inputs


def _op(L, U, kappa):
    V = int(np.prod(L))

    def f(Y):
        return oracle.apply_A(L, U, kappa, np.ascontiguousarray(Y).reshape(V, 4, 3, -1)).reshape(12 * V, -1)
    return f


def test_scalar_rational_function_on_a_diagonal_operator():
    rng = np.random.default_rng(11)
    n, m = 300, 3
    d = rng.uniform(0.05, 3.0, n)
    B = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    sig = np.array([1e-3, 0.02, 0.4, 2.5])
    coef = np.array([0.31, -1.7, 2.2, 0.05])
    c0 = 0.8
    r = oracle.dsbcg(lambda Y: d[:, None] * Y, B, sig, 1e-12)
    Y = oracle.partial_fraction(B, r.X, coef, c0)
    rat = c0 + sum(c / (sg + d) for c, sg in zip(coef, sig))
    exact = rat[:, None] * B
    assert np.linalg.norm(Y - exact) <= 1e-9 * np.linalg.norm(exact)


def test_product_identity_with_the_wilson_operator():
    L, kappa = (4, 4, 4, 4), 0.124
    U = inputs.make_links(L, "haar", inputs.rng_for(912, 0))
    V = int(np.prod(L))
    m = 2
    B = inputs.gaussian_rhs(inputs.rng_for(912, 1), V, m).reshape(12 * V, m)
    op = _op(L, U, kappa)
    s1, s2 = 0.01, 0.3
    r = oracle.dsbcg(op, B, [s1, s2], 1e-12)
    Y = oracle.partial_fraction(B, r.X, [1.0 / (s2 - s1), -1.0 / (s2 - s1)], 0.0)
    Z = op(Y) + s1 * Y
    back = op(Z) + s2 * Z
    # cond(s2 + A) * cond(s1 + A) bounds the amplification of the solve tolerance
    assert np.linalg.norm(back - B) <= 1e-7 * np.linalg.norm(B)
    # a sign or coefficient slip moves Y by O(1)
    Ybad = oracle.partial_fraction(B, r.X, [1.0 / (s2 - s1), 1.0 / (s2 - s1)], 0.0)
    Zb = op(Ybad) + s1 * Ybad
    assert np.linalg.norm(op(Zb) + s2 * Zb - B) > 1e-2 * np.linalg.norm(B)


@pytest.mark.parametrize("c0", [0.0, -2.5])
def test_limits(c0):
    rng = np.random.default_rng(3)
    B = rng.standard_normal((50, 2)) + 0j
    X = rng.standard_normal((3, 50, 2)) + 1j * rng.standard_normal((3, 50, 2))
    np.testing.assert_array_equal(oracle.partial_fraction(B, X, [0.0, 0.0, 0.0], c0), c0 * B)
    np.testing.assert_array_equal(oracle.partial_fraction(B, X[:1], [1.0], 0.0), X[0])
