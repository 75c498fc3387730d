"""DSBlockCG on the GPU against the CPU oracle.

FP64 form: iterate parity at a fixed number of block steps (<= 1e-10, expected
~1e-13), convergence to relative residual 1e-10 matching dense solves and the
oracle, deflation of duplicated right-hand sides, zero columns, the error
paths, determinism and the extreme sizes (m = s = 1, m = s = 16)."""
import numpy as np
import pytest

import oracle
from paper_1205_0359_amd import inputs
import paper_1205_0359_amd as dsb

from gpu_util import announce, dev, host, rel_fro, rel_max

pytestmark = pytest.mark.gpu


def _op(L, U, kappa):
    V = int(np.prod(L))

    def f(Y):
        return oracle.apply_A(L, U, kappa, np.ascontiguousarray(Y).reshape(V, 4, 3, -1)).reshape(12 * V, -1)
    return f


def _problem(L, m, seed, kind="haar", rhs="gaussian"):
    V = int(np.prod(L))
    U = inputs.make_links(L, kind, inputs.rng_for(seed, 0))
    if rhs == "deflating":
        B = inputs.deflating_rhs(inputs.rng_for(seed, 1), inputs.rng_for(seed, 2), V)
    else:
        B = inputs.make_rhs(rhs, V, m, inputs.rng_for(seed, 1))
    return U, B


def _gpu_solve(L, U, kappa, B, sig, tol, **kw):
    h = dsb.Handle(L)
    X, st = dsb.dsbcg_solve(h, dev(U), kappa, dev(B), sig, tol, **kw)
    return host(X), st


@pytest.mark.parametrize("L,m,sig,k,kind", [
    ((4, 4, 4, 4), 4, (1e-3, 1e-2, 1e-1), 12, "haar"),
    ((3, 4, 5, 6), 5, (1e-4, 0.3, 2.0, 0.05), 9, "smooth"),
    ((8, 6, 4, 10), 12, (1e-2,), 6, "haar"),
    ((4, 4, 4, 4), 1, (1e-3, 1e-1), 20, "smooth"),
])
def test_fixed_iteration_parity_fp64(L, m, sig, k, kind):
    announce("solve fixed", L, m, sig, k)
    kappa = 0.124
    U, B = _problem(L, m, 800 + m, kind)
    n = 12 * int(np.prod(L))
    ref = oracle.dsbcg(_op(L, U, kappa), B.reshape(n, m), sig, 1e-30, fixed_iters=k)
    X, st = _gpu_solve(L, U, kappa, B, sig, 1e-30, fixed_iters=k)
    assert st["block_iters"] == ref.iters and st["rank0"] == ref.rank0
    assert 0 <= st["qr2_skipped"] <= k
    for j in range(len(sig)):
        got = X[j].reshape(n, m)
        assert rel_fro(got, ref.X[j]) <= 1e-10, j
        assert rel_max(got, ref.X[j]) <= 1e-10, j
    np.testing.assert_allclose(st["est_relres"], ref.est, rtol=1e-8, atol=1e-14)


@pytest.mark.parametrize("window", [1, 3, 5])
def test_window_lengths_fixed_iterations(window):
    """Per-shift updates applied once per window of block steps (the last
    window ragged) give the oracle's step-wise iterates."""
    L, m, sig, k = (4, 4, 4, 6), 6, (1e-3, 3e-2, 0.5), 11
    announce("solve window", L, m, sig, k, window)
    kappa = 0.124
    U, B = _problem(L, m, 805, "haar")
    n = 12 * int(np.prod(L))
    ref = oracle.dsbcg(_op(L, U, kappa), B.reshape(n, m), sig, 1e-30, fixed_iters=k)
    X, st = _gpu_solve(L, U, kappa, B, sig, 1e-30, fixed_iters=k, window=window)
    for j in range(len(sig)):
        assert rel_fro(X[j].reshape(n, m), ref.X[j]) <= 1e-10, j
        assert rel_max(X[j].reshape(n, m), ref.X[j]) <= 1e-10, j


def test_window_with_freezing():
    """Shifts and columns that freeze inside a window: window lengths 1 and
    automatic agree, and every system meets the tolerance."""
    L, m = (4, 4, 4, 4), 5
    sig = (1e-3, 0.05, 0.8, 4.0)
    announce("solve window freezing", L, m, sig)
    U, B = _problem(L, m, 806, "smooth")
    B[..., 2] *= 1e-3  # a column with a much smaller norm converges on its own schedule
    X1, s1 = _gpu_solve(L, U, 0.125, B, sig, 1e-10, window=1)
    X0, s0 = _gpu_solve(L, U, 0.125, B, sig, 1e-10)
    assert s1["block_iters"] == s0["block_iters"]
    assert s0["true_relres"].max() <= 1e-10 and s1["true_relres"].max() <= 1e-10
    n = 12 * int(np.prod(L))
    for j in range(len(sig)):
        assert rel_fro(X0[j].reshape(n, m), X1[j].reshape(n, m)) <= 1e-11, j
    with pytest.raises(dsb.DSBCGError):
        _gpu_solve(L, U, 0.125, B, sig, 1e-10, window=-1)


def test_converges_to_dense_solution_4x4x4x4():
    w = inputs.WORKLOADS["haar4^4_m4_s3"]
    announce("solve converge", w.name)
    U, B = w.make()
    n, m = w.n, w.m
    op = _op(w.L, U, w.kappa)
    X, st = _gpu_solve(w.L, U, w.kappa, B, w.shifts, w.tol)
    assert st["status"] == "OK"
    Xs = X.reshape(len(w.shifts), n, m)
    tr = oracle.true_relres(op, B.reshape(n, m), w.shifts, Xs)
    assert tr.max() <= w.tol
    np.testing.assert_allclose(st["true_relres"], tr, rtol=1e-6, atol=1e-15)
    A = op(np.eye(n, dtype=complex))
    ev = np.linalg.eigvalsh(A)
    ref = oracle.dsbcg(op, B.reshape(n, m), w.shifts, w.tol)
    assert abs(st["block_iters"] - ref.iters) <= 1
    for j, sg in enumerate(w.shifts):
        dense = np.linalg.solve(A + sg * np.eye(n), B.reshape(n, m))
        cond = (ev[-1] + sg) / (ev[0] + sg)
        assert rel_fro(Xs[j], dense) <= cond * w.tol
        assert rel_fro(Xs[j], ref.X[j]) <= 2 * cond * w.tol


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (4, 4, 6, 8)])
def test_deflation_of_duplicated_columns(L):
    announce("solve deflating", L)
    kappa = 0.124
    U, B = _problem(L, 8, 830, "haar", "deflating")
    sig = tuple(np.logspace(-5, 0, 10))
    X, st = _gpu_solve(L, U, kappa, B, sig, 1e-10)
    assert st["rank0"] == 5 and st["status"] == "OK"
    assert st["true_relres"].max() <= 1e-10
    n = 12 * int(np.prod(L))
    tr = oracle.true_relres(_op(L, U, kappa), B.reshape(n, 8), sig, X.reshape(len(sig), n, 8))
    assert tr.max() <= 1e-10
    scale = np.abs(X).max()
    assert np.abs(X[..., 2] - X[..., 0]).max() <= 1e-13 * scale
    assert np.abs(X[..., 5] - X[..., 1]).max() <= 1e-13 * scale
    assert np.abs(X[..., 7] - X[..., 4]).max() <= 1e-9 * scale


def test_zero_columns_and_zero_rhs():
    L = (4, 4, 4, 4)
    announce("solve zero columns", L)
    U, B = _problem(L, 4, 840)
    B[..., 2] = 0
    X, st = _gpu_solve(L, U, 0.12, B, (1e-2, 1.0), 1e-10)
    assert st["rank0"] == 3
    assert np.all(X[..., 2] == 0)
    assert st["true_relres"][[0, 1, 3]].max() <= 1e-10
    X0, st0 = _gpu_solve(L, U, 0.12, np.zeros_like(B), (1e-2, 1.0), 1e-10)
    assert np.all(X0 == 0) and st0["block_iters"] == 0 and st0["rank0"] == 0


def test_not_hpd_and_not_converged():
    L = (4, 4, 4, 4)
    announce("solve error paths", L)
    U, B = _problem(L, 4, 850)
    with pytest.raises(dsb.NotHPDError):
        _gpu_solve(L, U, 0.12, B, (0.1, -10.0), 1e-10)
    h = dsb.Handle(L)
    X, st = dsb.dsbcg_solve(h, dev(U), 0.12, dev(B), (1e-2,), 1e-10, max_iters=3,
                            raise_not_converged=False)
    assert st["status"] == "ERR_NOT_CONVERGED" and st["block_iters"] == 3
    n = 12 * 256
    ref = oracle.dsbcg(_op(L, U, 0.12), B.reshape(n, 4), (1e-2,), 1e-10, fixed_iters=3)
    assert rel_fro(host(X)[0].reshape(n, 4), ref.X[0]) <= 1e-11
    with pytest.raises(dsb.NotConvergedError):
        dsb.dsbcg_solve(h, dev(U), 0.12, dev(B), (1e-2,), 1e-10, max_iters=3)
    with pytest.raises(dsb.DSBCGError):
        dsb.dsbcg_solve(h, dev(U), 0.12, dev(B), (float("inf"),), 1e-10)
    with pytest.raises(dsb.DSBCGError):
        dsb.dsbcg_solve(h, dev(U), 0.12, dev(B), (1e-2,), 0.0)
    Un = U.copy()
    Un[3, 1, 0, 0] = np.nan
    with pytest.raises(dsb.NotHPDError):
        dsb.dsbcg_solve(h, dev(Un), 0.12, dev(B), (1e-2,), 1e-10)
    Bn = B.copy()
    Bn[7, 0, 0, 1] = np.inf
    with pytest.raises(dsb.NotHPDError):
        dsb.dsbcg_solve(h, dev(U), 0.12, dev(Bn), (1e-2,), 1e-10)


def test_solve_repeatable_bitwise():
    L = (4, 4, 6, 8)
    announce("solve repeat", L)
    U, B = _problem(L, 6, 860, "smooth")
    h = dsb.Handle(L)
    dU, dB = dev(U), dev(B)
    X1, s1 = dsb.dsbcg_solve(h, dU, 0.125, dB, (1e-3, 1e-1), 1e-10)
    X2, s2 = dsb.dsbcg_solve(h, dU, 0.125, dB, (1e-3, 1e-1), 1e-10)
    assert np.array_equal(host(X1), host(X2)) and s1["block_iters"] == s2["block_iters"]


def test_profile_class_mask():
    """dsbcg_profile_select: with the mask of one class only that class's
    launches are timed (the others count none); with every class the totals
    match the selected class's, and the solution is the same bit for bit."""
    L = (4, 4, 6, 8)
    announce("profile mask", L)
    U, B = _problem(L, 5, 861, "smooth")
    h = dsb.Handle(L)
    dU, dB = dev(U), dev(B)
    names = [dsb.load().dsbcg_profile_name(k).decode() for k in range(32)
             if dsb.load().dsbcg_profile_name(k)]
    k = names.index("wilson_stencil.f64")
    dsb.dsbcg_profile_enable(h, True)
    X1, s1 = dsb.dsbcg_solve(h, dU, 0.125, dB, (1e-3, 1e-1), 1e-10)
    every = dsb.dsbcg_profile_read(h)
    dsb.dsbcg_profile_select(h, 1 << k)
    dsb.dsbcg_profile_enable(h, True)
    X2, s2 = dsb.dsbcg_solve(h, dU, 0.125, dB, (1e-3, 1e-1), 1e-10)
    one = dsb.dsbcg_profile_read(h)
    dsb.dsbcg_profile_enable(h, False)
    dsb.dsbcg_profile_select(h)
    assert np.array_equal(host(X1), host(X2))
    assert sum(v["launches"] > 0 for v in every.values()) >= 4
    for name, v in one.items():
        if name == "wilson_stencil.f64":
            assert v["launches"] == every[name]["launches"] > 0
            assert v["bytes"] == every[name]["bytes"] and v["ms"] > 0
        else:
            assert v["launches"] == 0 and v["ms"] == 0 and v["bytes"] == 0, name


@pytest.mark.parametrize("m,s", [(1, 1), (16, 16)])
def test_extreme_widths(m, s):
    L = (2, 2, 4, 4)
    announce("solve extreme widths", L, m, s)
    U, B = _problem(L, m, 870 + m, "smooth")
    sig = tuple(np.logspace(-3, 0, s))
    X, st = _gpu_solve(L, U, 0.125, B, sig, 1e-10)
    n = 12 * int(np.prod(L))
    tr = oracle.true_relres(_op(L, U, 0.125), B.reshape(n, m), sig, X.reshape(s, n, m))
    assert tr.max() <= 1e-10
    ref = oracle.dsbcg(_op(L, U, 0.125), B.reshape(n, m), sig, 1e-10)
    for j in range(s):
        assert rel_fro(X[j].reshape(n, m), ref.X[j]) <= 1e-6


def test_full_size_fp64_16x16x16x16():
    """The 16^4 smooth-link workload in FP64: every (l, j) converged to 1e-10; the
    oracle recomputes the residual of the two extreme shifts."""
    w = inputs.WORKLOADS["smooth16^4_m12_s8"]
    announce("solve full size", w.name)
    U, B = w.make()
    X, st = _gpu_solve(w.L, U, w.kappa, B, w.shifts, w.tol)
    assert st["status"] == "OK"
    assert st["true_relres"].max() <= w.tol
    op = _op(w.L, U, w.kappa)
    for j in (0, len(w.shifts) - 1):
        tr = oracle.true_relres(op, B.reshape(w.n, w.m), [w.shifts[j]], X[j].reshape(1, w.n, w.m))
        assert tr.max() <= w.tol
        np.testing.assert_allclose(tr[:, 0], st["true_relres"][:, j], rtol=1e-5)


@pytest.mark.parametrize("m,s,window", [(12, 10, 2), (16, 16, 3), (9, 13, 2)])
def test_wide_outputs_over_several_windows(m, s, window):
    """Windows that form P_{j,end} with wide outputs (m + b_end complex
    outputs: 3 or 4 matrix-core tiles) and more shifts than one launch takes
    (the shift set is split across launches), against the oracle's
    step-wise iterates at a fixed step count."""
    L, k = (4, 4, 4, 4), 7
    sig = tuple(np.logspace(-3, 0, s))
    announce("solve wide windows", L, m, s, window)
    kappa = 0.124
    U, B = _problem(L, m, 880 + m, "haar")
    n = 12 * int(np.prod(L))
    ref = oracle.dsbcg(_op(L, U, kappa), B.reshape(n, m), sig, 1e-30, fixed_iters=k)
    X, st = _gpu_solve(L, U, kappa, B, sig, 1e-30, fixed_iters=k, window=window)
    assert st["block_iters"] == k
    for j in range(s):
        assert rel_fro(X[j].reshape(n, m), ref.X[j]) <= 1e-10, j
        assert rel_max(X[j].reshape(n, m), ref.X[j]) <= 1e-10, j


def test_mvm_ordering_of_table_1_through_the_library():
    """The four methods of the paper's Table 1 (Sec. 4) as special cases of
    dsbcg_solve (m = 1: shifted CG; s = 1: block CG per shift; m = s = 1: CG)
    on a near-critical 3^4 field of the table's shape: every run converges,
    takes the oracle's block-step count to within one step, and the mvm
    totals are ordered as in the table."""
    L, kappa, m = (3, 3, 3, 3), 0.125, 4
    announce("table 1 ordering", L)
    V = int(np.prod(L))
    n = 12 * V
    U = inputs.make_links(L, "smooth", inputs.rng_for(990, 0))
    B = inputs.gaussian_rhs(inputs.rng_for(990, 1), V, m)
    sig = tuple(np.logspace(-6, -1, 7))
    tol = 1e-8
    op = _op(L, U, kappa)
    Bn = B.reshape(n, m)
    h = dsb.Handle(L)
    dU = dev(U)
    cases = {
        "DSBlockCG": [(list(range(m)), sig)],
        "shiftedCG": [([l], sig) for l in range(m)],
        "BlockCG": [(list(range(m)), (s,)) for s in sig],
        "CG": [([l], (s,)) for l in range(m) for s in sig],
    }
    totals = {}
    for name, runs in cases.items():
        tot = 0
        for cols, sh in runs:
            Bc = np.ascontiguousarray(B[..., cols])
            X, st = dsb.dsbcg_solve(h, dU, kappa, dev(Bc), sh, tol)
            assert st["status"] == "OK" and st["true_relres"].max() <= tol, (name, cols, sh)
            ref = oracle.dsbcg(op, np.ascontiguousarray(Bn[:, cols]), sh, tol)
            assert abs(st["block_iters"] - ref.iters) <= 1, (name, cols, sh, st["block_iters"], ref.iters)
            tot += st["mvms"]
        totals[name] = tot
    order = ("DSBlockCG", "shiftedCG", "BlockCG", "CG")
    got = [totals[k] for k in order]
    print("mvms", totals)
    assert got == sorted(got) and len(set(got)) == 4
    assert got[0] / got[1] < 0.8


def test_fp64_form_full_size_32x32x32x64():
    """The 32^3 x 64 workload (m = 8 of rank 5, 10 shifts) in the FP64 form,
    as the benchmark times it: every (l, j) reaches the FP64 true residual
    1e-10, the duplicated right-hand sides give equal solution columns, and
    the oracle evaluates b - (sigma_j + A) x_j at sampled sites for the
    smallest and largest shift (restricted to those sites it is at most
    tol ||b_l||)."""
    w = inputs.WORKLOADS["haar32^3x64_m8r5_s10"]
    announce("fp64 form full size", w.name)
    U, B = w.make()
    h = dsb.Handle(w.L)
    X, st = dsb.dsbcg_solve(h, dev(U), w.kappa, dev(B), w.shifts, w.tol)
    assert st["status"] == "OK" and st["rank0"] == 5
    assert st["true_relres"].max() <= w.tol
    h.close()  # the handle keeps most of the free memory as its workspace
    for j in range(len(w.shifts)):
        scale = float(X[j].abs().max())
        assert float((X[j][..., 2] - X[j][..., 0]).abs().max()) <= 1e-13 * scale, j
        assert float((X[j][..., 5] - X[j][..., 1]).abs().max()) <= 1e-13 * scale, j
    rng = np.random.default_rng(8)
    sites = np.concatenate([[0, w.V - 1], rng.integers(0, w.V, 30)])
    bnorm = np.linalg.norm(B.reshape(-1, w.m), axis=0)
    for j in (0, len(w.shifts) - 1):
        Xh = host(X[j])
        AX = oracle.apply_A_sites(w.L, U, w.kappa, Xh, sites)
        R = B[sites] - w.shifts[j] * Xh[sites] - AX
        on_sites = np.sqrt((np.abs(R) ** 2).sum(axis=(0, 1, 2)))
        assert np.all(on_sites <= w.tol * bnorm), j
        del Xh


def test_workspace_kept_by_default_and_released_on_request():
    """A solve with keep_workspace = 0 frees its device workspace at return; by
    default the handle keeps it, and dsbcg_release_workspace frees it.  The
    results are the same."""
    import torch
    w = inputs.WORKLOADS["smooth16^4_m4_s6_grad"]
    announce("workspace", w.name)
    U, B = w.make()
    h = dsb.Handle(w.L)
    dU, dB = dev(U), dev(B)
    dsb.dsbcg_stage_links(h, dU)
    X = torch.empty((len(w.shifts), w.V, 4, 3, w.m), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    X1, s1 = dsb.dsbcg_solve(h, None, w.kappa, dB, w.shifts, w.tol, X=X, keep_workspace=0)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    x1 = host(X1).copy()
    X2, s2 = dsb.dsbcg_solve(h, None, w.kappa, dB, w.shifts, w.tol, X=X)
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    assert np.array_equal(host(X2), x1) and s1["block_iters"] == s2["block_iters"]
    dsb.dsbcg_release_workspace(h)
    torch.cuda.synchronize()
    free3 = torch.cuda.mem_get_info()[0]
    # the iterates alone are s * 12 V m complex128 = 201 MB
    held = 12 * w.V * w.m * len(w.shifts) * 16
    assert free0 - free1 < 64 << 20, (free0, free1)
    assert free1 - free2 > held, (free1, free2)
    assert free0 - free3 < 64 << 20, (free0, free3)


def test_residual_history_matches_oracle():
    """stats.est_history: after each main-phase step, the largest estimated
    relative residual over the systems updated in that step, against the
    oracle's per-step estimates (systems active in step i: not frozen before
    it).  tol 1e-6 over 30 fixed steps: the shifts freeze at steps 22, 26
    and 27, the last steps update nothing (history 0)."""
    w = inputs.WORKLOADS["haar4^4_m4_s3"]
    announce("residual history", w.name)
    U, B = w.make()
    n, m = w.n, w.m
    X, st = _gpu_solve(w.L, U, w.kappa, B, w.shifts, 1e-6, fixed_iters=30)
    ref = oracle.dsbcg(_op(w.L, U, w.kappa), B.reshape(n, m), w.shifts, 1e-6, fixed_iters=30)
    hist = st["est_history"]
    assert len(hist) == ref.iters == 30
    assert np.array_equal(np.unique(ref.frozen_at), [22, 26, 27])
    for i in range(1, ref.iters + 1):
        act = (ref.frozen_at == -1) | (ref.frozen_at >= i)
        want = ref.history[i - 1][act].max() if act.any() else 0.0
        assert abs(hist[i - 1] - want) <= 1e-6 * want, (i, hist[i - 1], want)
    assert hist[26] <= 1e-6 < hist[0] and hist[27:] == [0.0, 0.0, 0.0]
