"""Link-derivative stencil on the GPU against the oracle's (which is pinned by
finite differences in the CPU tests)."""
import numpy as np
import pytest

import oracle
from paper_1205_0359_amd import inputs
import paper_1205_0359_amd as dsb

from gpu_util import announce, dev, host, rel_max

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,k", [((4, 4, 4, 4), 1), ((3, 4, 5, 6), 5), ((8, 6, 4, 10), 20)])
def test_link_grad_matches_oracle(L, k):
    announce("link_grad", L, k)
    V = int(np.prod(L))
    U = inputs.make_links(L, "haar", inputs.rng_for(890, 0))
    phi = inputs.gaussian_rhs(inputs.rng_for(890, 1), V, k)
    psi = inputs.gaussian_rhs(inputs.rng_for(890, 2), V, k)
    h = dsb.Handle(L)
    G = host(dsb.dsbcg_link_grad(h, 0.13, dev(phi), dev(psi)))
    want = oracle.link_grad(L, 0.13, phi, psi)
    assert rel_max(G, want) <= 1e-13
    del U


def _op(L, U, kappa):
    V = int(np.prod(L))

    def f(Y):
        return oracle.apply_A(L, U, kappa, np.ascontiguousarray(Y).reshape(V, 4, 3, -1)).reshape(12 * V, -1)
    return f


def test_solve_multi_per_shift_right_hand_sides():
    L = (4, 4, 4, 4)
    announce("solve_multi", L)
    V, m = 256, 3
    U = inputs.make_links(L, "haar", inputs.rng_for(891, 0))
    sig = (1e-3, 0.1, 1.0)
    G = inputs.complex_gaussian(inputs.rng_for(891, 1), (len(sig), V, 4, 3, m))
    h = dsb.Handle(L)
    Lam, st = dsb.dsbcg_solve_multi(h, dev(U), 0.12, dev(G), sig, 1e-11)
    assert st["rank0"] == 9 and st["true_relres"].max() <= 1e-11
    Lh = host(Lam)
    op = _op(L, U, 0.12)
    for j, sg in enumerate(sig):
        ref = oracle.dsbcg(op, G[j].reshape(-1, m), [sg], 1e-12)
        assert np.linalg.norm(Lh[j].reshape(-1, m) - ref.X[0]) <= 1e-9 * np.linalg.norm(ref.X[0])
    # blocks proportional to one B: a single basis of width m
    B = inputs.gaussian_rhs(inputs.rng_for(891, 2), V, m)
    Gp = np.stack([a * B for a in (0.3, -1.2, 2.0)])
    Lp, st = dsb.dsbcg_solve_multi(h, dev(U), 0.12, dev(Gp), sig, 1e-11)
    assert st["rank0"] == m
    X, _ = dsb.dsbcg_solve(h, dev(U), 0.12, dev(B), sig, 1e-11)
    for j, a in enumerate((0.3, -1.2, 2.0)):
        assert rel_max(host(Lp)[j], a * host(X)[j]) <= 1e-9


def _trace_loss_setup(L, kappa, seed, prec):
    import torch
    from paper_1205_0359_amd.autograd import solve
    V = int(np.prod(L))
    U = inputs.make_links(L, "haar", inputs.rng_for(seed, 0))
    B = inputs.gaussian_rhs(inputs.rng_for(seed, 1), V, 4)
    sig = np.logspace(-3, 0, 6)
    alpha = inputs.rng_for(seed, 2).uniform(0.1, 1.0, 6)
    h = dsb.Handle(L)
    tU = dev(U).requires_grad_(True)
    tB = dev(B).requires_grad_(True)
    ts = torch.tensor(sig, dtype=torch.float64, requires_grad=True)
    X = solve(tU, tB, ts, h, kappa, 1e-11, precision=prec)
    ta = dev(alpha)
    loss = sum(ta[j] * (tB.conj() * X[j]).sum().real for j in range(6))
    loss.backward()
    return U, B, sig, alpha, X.detach(), tU.grad, tB.grad, ts.grad, h


@pytest.mark.parametrize("prec", [dsb.DSBCG_FP64, dsb.DSBCG_FP32_RELIABLE])
def test_autograd_trace_loss_against_oracle(prec):
    L, kappa = (4, 4, 4, 4), 0.12
    announce("autograd trace loss", L, prec)
    U, B, sig, alpha, X, gU, gB, gs, h = _trace_loss_setup(L, kappa, 892, prec)
    Xh = host(X)
    want_B = 2 * sum(alpha[j] * Xh[j] for j in range(6))
    assert rel_max(host(gB), want_B) <= 1e-8
    want_s = np.array([-alpha[j] * np.linalg.norm(Xh[j]) ** 2 for j in range(6)])
    assert np.allclose(gs.numpy(), want_s, rtol=1e-8)
    op = _op(L, U, kappa)
    Xo = np.stack([oracle.dsbcg(op, B.reshape(-1, 4), [sg], 1e-12).X[0].reshape(B.shape) for sg in sig])
    G = np.stack([alpha[j] * B for j in range(6)])
    dU, _, _, _ = oracle.adjoint_gradients(L, U, kappa, B, sig, Xo, G, tol=1e-12)
    assert rel_max(host(gU), dU) <= 1e-8


def test_autograd_link_gradient_finite_differences():
    """Central differences of the loss on 32 random link entries (real or imaginary
    part), each loss evaluated with FP64 solves to 1e-13."""
    import torch
    L, kappa = (4, 4, 4, 4), 0.12
    announce("autograd FD", L)
    U, B, sig, alpha, X, gU, gB, gs, h = _trace_loss_setup(L, kappa, 893, dsb.DSBCG_FP64)
    gUh = host(gU)
    dB = dev(B)

    def loss(Uv):
        Xv, _ = dsb.dsbcg_solve(h, dev(Uv), kappa, dB, sig, 1e-13)
        Xv = host(Xv)
        return sum(alpha[j] * np.vdot(B.ravel(), Xv[j].ravel()).real for j in range(6))

    rng = inputs.rng_for(893, 3)
    eps = 1e-5
    for _ in range(32):
        idx = (rng.integers(0, 256), rng.integers(0, 4), rng.integers(0, 3), rng.integers(0, 3))
        unit = 1.0 if rng.integers(0, 2) == 0 else 1j
        Up, Um = U.copy(), U.copy()
        Up[idx] += eps * unit
        Um[idx] -= eps * unit
        fd = (loss(Up) - loss(Um)) / (2 * eps)
        an = gUh[idx].real if unit == 1.0 else gUh[idx].imag
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (idx, unit, fd, an)
    del torch


def test_autograd_recompute_matches_stored():
    import torch
    from paper_1205_0359_amd.autograd import solve
    L, kappa = (4, 4, 4, 8), 0.124
    announce("autograd recompute", L)
    V = int(np.prod(L))
    U = inputs.make_links(L, "haar", inputs.rng_for(894, 0))
    B = inputs.gaussian_rhs(inputs.rng_for(894, 1), V, 3)
    sig = np.logspace(-4, 0, 4)
    grads = []
    h = dsb.Handle(L)
    for rec in (False, True):
        tU = dev(U).requires_grad_(True)
        tB = dev(B).requires_grad_(True)
        ts = torch.tensor(sig, dtype=torch.float64, requires_grad=True)
        X = solve(tU, tB, ts, h, kappa, 1e-11, recompute=rec)
        (X.abs() ** 2).sum().backward()
        grads.append((host(tU.grad), host(tB.grad), ts.grad.numpy()))
    for a, b in zip(*grads):
        assert np.array_equal(a, b)
