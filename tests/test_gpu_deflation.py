"""Deflation inside the iteration on the GPU against the oracle.

A new Lanczos direction that depends linearly on the earlier blocks is
dropped (Sec. 1: deflation guarantees convergence; Sec. 3: once it happens
the block width, and with it the bandwidth of T, shrinks).  The cases:

* B = [b1 | A b1 | b3 | b4], as given and rotated by a random 4 x 4 unitary:
  span(A V_1) meets span(V_1) in one direction, so the second block has
  width 3.  Rotated, no column of W is small and the dependence shows only
  in the last Schur remainder of W^H W, below what the Cholesky QR resolves:
  the step's QR is redone column by column.
* Plane waves at unit links (eigenvectors of A): the space of B is invariant,
  the first step exhausts it, X_j = b / (sigma_j + lambda(p)).
* Two plane waves per column with different eigenvalues: the block Krylov
  space has dimension 2m, the second step exhausts it, and X_j is exact.
* 2^4 lattice (n = 192): the block Krylov space fills the whole space.

FP64 and the partial-fraction form at a fixed step count against the
oracle, element-wise (max |difference| / max |oracle|) and by norm at 1e-10
(expected ~1e-13), with equal widths step by step.  The FP32 form with FP32
vectors from the first step drops the same directions (widths equal to the
oracle's) and converges to the FP64 true residual 1e-10."""
import numpy as np
import pytest

import oracle
from paper_1205_0359_amd import inputs
import paper_1205_0359_amd as dsb

from gpu_util import announce, dev, host, rel_fro, rel_max

pytestmark = pytest.mark.gpu

L4 = (4, 4, 4, 4)
KAPPA = 0.124
SIG = (1e-3, 2e-2, 0.4)
COEF = (0.6, -1.3, 2.1)
C0 = 0.25


def _op(L, U, kappa):
    V = int(np.prod(L))

    def f(Y):
        return oracle.apply_A(L, U, kappa, np.ascontiguousarray(Y).reshape(V, 4, 3, -1)).reshape(12 * V, -1)
    return f


def _dependent_rhs(seed, rotate):
    """[b1 | A b1 | b3 | b4] (A from the oracle), optionally times a random unitary."""
    V = int(np.prod(L4))
    U = inputs.make_links(L4, "haar", inputs.rng_for(seed, 0))
    G = inputs.gaussian_rhs(inputs.rng_for(seed, 1), V, 3)
    b1 = G[..., 0:1]
    Ab1 = oracle.apply_A(L4, U, KAPPA, np.ascontiguousarray(b1))
    B = np.concatenate([b1, Ab1, G[..., 1:3]], axis=-1)
    if rotate:
        Z = inputs.complex_gaussian(inputs.rng_for(seed, 3), (4, 4))
        Q, R = np.linalg.qr(Z)
        B = B @ Q
    return U, np.ascontiguousarray(B)


def _lam(L, nvec, kappa):
    """Eigenvalue of A = D^H D on the plane wave of momentum 2 pi nvec / L at unit links."""
    p = 2 * np.pi * np.asarray(nvec) / np.asarray(L)
    a = 1 - 2 * kappa * np.cos(p).sum()
    return a * a + 4 * kappa ** 2 * (np.sin(p) ** 2).sum()


def _solve(L, U, B, sig, tol, **kw):
    h = dsb.Handle(L)
    X, st = dsb.dsbcg_solve(h, dev(U), KAPPA, dev(B), sig, tol, **kw)
    return host(X), st


def _rational(L, U, B, sig, tol, **kw):
    h = dsb.Handle(L)
    Y, st = dsb.dsbcg_solve_rational(h, dev(U), KAPPA, dev(B), sig, COEF[:len(sig)], C0, tol, **kw)
    return host(Y), st


@pytest.mark.parametrize("rotate", [False, True])
@pytest.mark.parametrize("window", [0, 1])
def test_dependent_direction_fp64_fixed_steps(rotate, window):
    k = 8
    announce("deflation fp64", "rotate", rotate, "window", window, "k", k)
    U, B = _dependent_rhs(1100, rotate)
    n, m = B.shape[0] * 12, 4
    ref = oracle.dsbcg(_op(L4, U, KAPPA), B.reshape(n, m), SIG, 1e-30, fixed_iters=k, record=True)
    assert ref.widths[:2] == [4, 3]  # the oracle drops exactly one direction at step 1
    X, st = _solve(L4, U, B, SIG, 1e-30, fixed_iters=k, window=window)
    assert st["widths"] == ref.widths
    final = ref.Vs[-1].shape[1]  # width of V_{k+1}
    assert st["final_width"] == final and st["deflations"] == ref.widths[0] - final
    assert st["mvms"] == ref.mvms
    if rotate:
        assert st["qr_redone"] >= 1  # decided column by column, not by the Gram matrix
    for j in range(len(SIG)):
        got = X[j].reshape(n, m)
        assert rel_fro(got, ref.X[j]) <= 1e-10, j
        assert rel_max(got, ref.X[j]) <= 1e-10, j
    np.testing.assert_allclose(st["est_relres"], ref.est, rtol=1e-8, atol=1e-14)


@pytest.mark.parametrize("rotate", [False, True])
def test_dependent_direction_rational_fixed_steps(rotate):
    k = 8
    announce("deflation rational", "rotate", rotate, "k", k)
    U, B = _dependent_rhs(1101, rotate)
    n, m = B.shape[0] * 12, 4
    ref = oracle.dsbcg(_op(L4, U, KAPPA), B.reshape(n, m), SIG, 1e-30, fixed_iters=k)
    assert ref.widths[:2] == [4, 3]
    want = oracle.partial_fraction(B.reshape(n, m), ref.X, COEF, C0)
    Y, st = _rational(L4, U, B, SIG, 1e-30, fixed_iters=k)
    assert st["widths"] == ref.widths and st["mvms"] == ref.mvms
    got = Y.reshape(n, m)
    assert rel_fro(got, want) <= 1e-10
    assert rel_max(got, want) <= 1e-10


@pytest.mark.parametrize("rotate", [False, True])
def test_dependent_direction_fp32_form(rotate):
    """FP32 vectors from the first step (switch_at = 2, above the initial estimates of 1): the direction is
    dropped in FP32 as in the oracle, and the solve meets the FP64 true
    residual tol."""
    announce("deflation fp32", "rotate", rotate)
    U, B = _dependent_rhs(1102, rotate)
    n, m = B.shape[0] * 12, 4
    k = 8
    ref = oracle.dsbcg(_op(L4, U, KAPPA), B.reshape(n, m), SIG, 1e-30, fixed_iters=k)
    X, st = _solve(L4, U, B, SIG, 1e-30, fixed_iters=k, precision=1, switch_at=2.0)
    assert st["switch_iter"] == 1
    assert st["widths"] == ref.widths
    for j in range(len(SIG)):
        # FP32 Lanczos vectors: rounding amplified by the conditioning of T_k
        assert rel_fro(X[j].reshape(n, m), ref.X[j]) <= 1e-4, j
    X, st = _solve(L4, U, B, SIG, 1e-10, precision=1, switch_at=2.0)
    assert st["widths"][:2] == [4, 3] and st["deflations"] >= 1
    assert st["true_relres"].max() <= 1e-10
    tr = oracle.true_relres(_op(L4, U, KAPPA), B.reshape(n, m), SIG, X.reshape(len(SIG), n, m))
    assert tr.max() <= 1e-10


def _plane_waves(L, momenta, seed):
    rng = inputs.rng_for(seed, 1)
    cols = [inputs.plane_wave(L, p, inputs.complex_gaussian(rng, (4, 3))) for p in momenta]
    return np.ascontiguousarray(np.stack(cols, axis=-1))


@pytest.mark.parametrize("form", ["fp64", "fp32", "rational"])
def test_plane_waves_exhaust_after_one_step(form):
    announce("deflation plane waves", form)
    momenta = ([1, 0, 0, 0], [0, 2, 1, 0], [3, 1, 0, 2])
    U = inputs.unit_links(L4)
    B = _plane_waves(L4, momenta, 1103)
    lams = np.array([_lam(L4, p, KAPPA) for p in momenta])
    sig = (1e-3, 0.5)
    want = np.stack([B / (sg + lams) for sg in sig])  # (s, V, 4, 3, m)
    if form == "rational":
        Y, st = _rational(L4, U, B, sig, 1e-10)
        exp = C0 * B + sum(c * want[j] for j, c in enumerate(COEF[:2]))
        assert rel_max(Y, exp) <= 1e-13
    else:
        X, st = _solve(L4, U, B, sig, 1e-10, precision=0 if form == "fp64" else 1)
        assert rel_max(X, want) <= 1e-13
        assert st["true_relres"].max() <= 1e-12
    assert st["block_iters"] == 1 and st["widths"] == [3]
    assert st["final_width"] == 0 and st["deflations"] == 3


@pytest.mark.parametrize("form", ["fp64", "fp32", "rational"])
def test_two_eigencomponents_exhaust_after_two_steps(form):
    """b_l = e^{i p_l x} chi_l + e^{i q_l x} chi'_l with lambda(p_l) != lambda(q_l):
    span{B, A B} is invariant, so the second step exhausts it and the
    iterates are exact."""
    announce("deflation two eigencomponents", form)
    P = ([1, 0, 0, 0], [0, 1, 1, 0], [2, 2, 0, 1])
    Qm = ([0, 0, 2, 0], [1, 1, 1, 1], [3, 0, 0, 0])
    U = inputs.unit_links(L4)
    E1 = _plane_waves(L4, P, 1104)
    E2 = _plane_waves(L4, Qm, 1105)
    B = E1 + E2
    l1 = np.array([_lam(L4, p, KAPPA) for p in P])
    l2 = np.array([_lam(L4, q, KAPPA) for q in Qm])
    assert np.all(np.abs(l1 - l2) > 1e-2)
    sig = (1e-3, 0.2, 1.5)
    want = np.stack([E1 / (sg + l1) + E2 / (sg + l2) for sg in sig])
    if form == "rational":
        Y, st = _rational(L4, U, B, sig, 1e-10)
        exp = C0 * B + sum(c * want[j] for j, c in enumerate(COEF))
        assert rel_max(Y, exp) <= 1e-12
    else:
        X, st = _solve(L4, U, B, sig, 1e-10, precision=0 if form == "fp64" else 1)
        assert rel_max(X, want) <= 1e-12
        assert st["true_relres"].max() <= 1e-10
    assert st["widths"] == [3, 3] and st["final_width"] == 0 and st["deflations"] == 3


def test_finite_termination_2x2x2x2():
    """n = 192: the block Krylov space fills the whole space; the GPU run
    follows the oracle's widths and step count and meets the dense solution."""
    L = (2, 2, 2, 2)
    announce("deflation 2^4 termination", L)
    U = inputs.make_links(L, "smooth", inputs.rng_for(906, 0), 0.3)
    B = inputs.gaussian_rhs(inputs.rng_for(906, 1), 16, 4)
    sig = (1e-4, 1e-1)
    op = _op(L, U, 0.125)
    n, m = 192, 4
    ref = oracle.dsbcg(op, B.reshape(n, m), sig, 1e-10)
    h = dsb.Handle(L)
    X, st = dsb.dsbcg_solve(h, dev(U), 0.125, dev(B), sig, 1e-10)
    X = host(X)
    assert abs(st["block_iters"] - ref.iters) <= 2
    assert st["widths"][:10] == ref.widths[:10]
    assert st["true_relres"].max() <= 1e-10
    A = op(np.eye(n, dtype=complex))
    ev = np.linalg.eigvalsh(A)
    for j, sg in enumerate(sig):
        dense = np.linalg.solve(A + sg * np.eye(n), B.reshape(n, m))
        cond = (ev[-1] + sg) / (ev[0] + sg)
        assert rel_fro(X[j].reshape(n, m), dense) <= cond * 1e-10
