"""Pins of the oracle's vector-wise stopping (Sec. 3) against facts fixed outside it.

Checked: the stage iterates equal the paper's scalar update
X^(k) = X^(k-1) + p^(k) u^(k) / d^(k) from a root-free Cholesky L D L^H of
T_sigma written out here; the stage residual norms ||C^(k)[:, l]|| equal the
true residuals ||b_l - (sigma + A) x_l^(k)|| (the residual paragraph of
Sec. 3); at block boundaries the stages equal the block form; each system
stops at the first stage whose Galerkin iterate -- formed here by projecting
(sigma + A) onto the basis with the operator itself, not from T -- has a
relative residual <= tol; m = 1 reduces to the block form; duplicated
columns stop together.
"""
import numpy as np
import pytest

import oracle
from paper_1205_0359_amd import inputs


def _op(L, U, kappa):
    V = int(np.prod(L))
    n = 12 * V

    def f(Y):
        return oracle.apply_A(L, U, kappa, np.ascontiguousarray(Y).reshape(V, 4, 3, -1)).reshape(n, -1)
    return f


@pytest.fixture(scope="module")
def small():
    w = inputs.WORKLOADS["haar4^4_m4_s3"]
    U, B = w.make()
    return w, B.reshape(w.n, w.m), _op(w.L, U, w.kappa)


@pytest.fixture(scope="module")
def recorded(small):
    w, B, op = small
    r = oracle.dsbcg_vectorwise(op, B, w.shifts, 1e-30, max_iters=6, record=True)
    return r


def _ldl(Ts):
    """Root-free Cholesky Ts = L D L^H (L unit lower, D real diagonal), scalar loops."""
    k = Ts.shape[0]
    L = np.eye(k, dtype=np.complex128)
    d = np.zeros(k)
    for c in range(k):
        d[c] = (Ts[c, c] - np.sum(np.abs(L[c, :c]) ** 2 * d[:c])).real
        for r in range(c + 1, k):
            L[r, c] = (Ts[r, c] - np.sum(L[r, :c] * d[:c] * L[c, :c].conj())) / d[c]
    return L, d


def test_stage_iterates_follow_the_scalar_update(small, recorded):
    w, B, op = small
    r = recorded
    K = sum(r.widths)
    V = r.Vall[:, :K]
    rho = oracle.deflated_qr(B, 0.1 * 1e-30 * np.linalg.norm(B, axis=0))[1]
    for sg in w.shifts:
        Ts = r.T[:K, :K] + sg * np.eye(K)
        L, d = _ldl(Ts)
        P = np.linalg.solve(L.conj(), V.T).T          # V L^{-H}: columns p^(k)
        E = np.zeros((K, w.m), dtype=np.complex128)
        E[:rho.shape[0]] = rho
        Uu = np.linalg.solve(L, E)                     # rows u^(k)
        X = np.zeros((w.n, w.m), dtype=np.complex128)
        for k in range(1, K + 1):
            X = X + np.outer(P[:, k - 1], Uu[k - 1]) / d[k - 1]
            Y, _ = oracle.stage_solution(r.T, rho, sg, k, r.known)
            Xk = V[:, :k] @ Y
            assert np.linalg.norm(X - Xk) <= 1e-12 * np.linalg.norm(Xk)


def test_stage_estimates_are_true_residuals(small, recorded):
    w, B, op = small
    r = recorded
    rho = oracle.deflated_qr(B, 0.0)[1]
    bn = np.linalg.norm(B, axis=0)
    for k in (1, 2, 3, 5, 7, 10, 13, 18):
        for sg in w.shifts:
            Y, C = oracle.stage_solution(r.T, rho, sg, k, r.known)
            X = r.Vall[:, :k] @ Y
            true = np.linalg.norm(B - sg * X - op(X), axis=0) / bn
            est = np.linalg.norm(C, axis=0) / bn
            assert np.allclose(est, true, rtol=1e-8, atol=1e-14), (k, sg)


def test_block_boundaries_equal_the_block_form(small, recorded):
    w, B, op = small
    r = recorded
    rho = oracle.deflated_qr(B, 0.0)[1]
    for i in (1, 2, 4, 5):
        blk = oracle.dsbcg(op, B, w.shifts, 1e-30, fixed_iters=i, freeze=False)
        k = sum(r.widths[:i])
        for j, sg in enumerate(w.shifts):
            Y, C = oracle.stage_solution(r.T, rho, sg, k, r.known)
            X = r.Vall[:, :k] @ Y
            assert np.linalg.norm(X - blk.X[j]) <= 1e-12 * np.linalg.norm(blk.X[j])
            est = np.linalg.norm(C, axis=0) / np.linalg.norm(B, axis=0)
            assert np.allclose(est, blk.est[:, j], rtol=1e-9, atol=1e-15)


@pytest.mark.parametrize("tol", [1e-4, 1e-10])
def test_each_system_stops_at_its_first_stage_below_tol(small, tol):
    w, B, op = small
    r = oracle.dsbcg_vectorwise(op, B, w.shifts, tol, record=True)
    bn = np.linalg.norm(B, axis=0)
    assert (r.frozen_stage > 0).all()
    assert r.mvms_vector == r.frozen_stage.max()
    assert r.mvms - r.widths[-1] < r.mvms_vector <= r.mvms

    def galerkin(k, sg, l):
        # Galerkin iterate on the first k basis vectors, projected with the operator
        Vk = r.Vall[:, :k]
        Ak = Vk.conj().T @ (op(Vk) + sg * Vk)
        x = Vk @ np.linalg.solve(Ak, Vk.conj().T @ B[:, l])
        return x, np.linalg.norm(B[:, l] - sg * x - op(x[:, None])[:, 0]) / bn[l]

    for j, sg in enumerate(w.shifts):
        for l in range(w.m):
            k = int(r.frozen_stage[l, j])
            x, res = galerkin(k, sg, l)
            assert res <= tol * (1 + 1e-6)
            assert np.linalg.norm(r.X[j][:, l] - x) <= 1e-9 * np.linalg.norm(x)
            if k > 1:
                _, res_prev = galerkin(k - 1, sg, l)
                assert res_prev > tol * (1 + 1e-6), (l, j, k)


def test_single_rhs_reduces_to_the_block_form(small):
    w, B, op = small
    b = B[:, 2:3]
    tol = 1e-10
    v = oracle.dsbcg_vectorwise(op, b, w.shifts, tol)
    blk = oracle.dsbcg(op, b, w.shifts, tol)
    assert np.array_equal(v.frozen_stage, blk.frozen_at)
    for j in range(len(w.shifts)):
        assert np.linalg.norm(v.X[j] - blk.X[j]) <= 1e-12 * np.linalg.norm(blk.X[j])


def test_duplicated_columns_stop_together(small):
    w, B, op = small
    Bd = np.concatenate([B[:, :3], B[:, :1]], axis=1)
    r = oracle.dsbcg_vectorwise(op, Bd, w.shifts, 1e-10)
    assert r.rank0 == 3
    assert np.array_equal(r.frozen_stage[3], r.frozen_stage[0])
    for j in range(len(w.shifts)):
        assert np.linalg.norm(r.X[j][:, 3] - r.X[j][:, 0]) <= 1e-13 * np.linalg.norm(r.X[j][:, 0])
