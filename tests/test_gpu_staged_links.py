"""Links staged once per handle (dsbcg_stage_links): calls with U = NULL give
the same results, bit for bit, as the same calls passing U; a later call with
another U replaces the staged copy; non-finite links are refused."""
import numpy as np
import pytest

import oracle
from paper_1205_0359_amd import inputs
import paper_1205_0359_amd as dsb

from gpu_util import announce, dev, host, rel_max

pytestmark = pytest.mark.gpu

L = (4, 6, 4, 6)
KAPPA = 0.124


def _case(m, seed):
    U = inputs.make_links(L, "haar", inputs.rng_for(seed, 0))
    X = inputs.gaussian_rhs(inputs.rng_for(seed, 1), int(np.prod(L)), m)
    return U, X


@pytest.mark.parametrize("m,precision", [(5, 0), (3, 0), (8, 0), (5, 1)])
def test_apply_with_staged_links_is_bitwise_equal(m, precision):
    announce("staged apply", L, m, precision)
    U, X = _case(m, 1200 + m)
    h = dsb.Handle(L)
    dU, dX = dev(U), dev(X)
    want = host(dsb.dsbcg_apply_A(h, dU, KAPPA, dX, precision=precision))
    dsb.dsbcg_stage_links(h, dU)
    got = host(dsb.dsbcg_apply_A(h, None, KAPPA, dX, precision=precision))
    assert np.array_equal(got, want)
    if precision == 0:
        assert rel_max(got, oracle.apply_A(L, U, KAPPA, X)) <= 1e-13
        for dag in (False, True):
            a = host(dsb.dsbcg_apply_D(h, None, KAPPA, dX, dagger=dag))
            b = host(dsb.dsbcg_apply_D(dsb.Handle(L), dU, KAPPA, dX, dagger=dag))
            assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_with_staged_links_is_bitwise_equal(precision):
    announce("staged solve", L, precision)
    U, B = _case(4, 1210)
    sig = (1e-3, 0.1)
    h = dsb.Handle(L)
    dU, dB = dev(U), dev(B)
    X1, s1 = dsb.dsbcg_solve(h, dU, KAPPA, dB, sig, 1e-10, precision=precision)
    h2 = dsb.Handle(L)
    dsb.dsbcg_stage_links(h2, dU)
    X2, s2 = dsb.dsbcg_solve(h2, None, KAPPA, dB, sig, 1e-10, precision=precision)
    assert np.array_equal(host(X1), host(X2))
    assert s1["block_iters"] == s2["block_iters"] and s2["true_relres"].max() <= 1e-10


def test_another_U_replaces_the_staged_copy_and_nan_is_refused():
    announce("staged replace", L)
    U, X = _case(2, 1220)
    U2 = inputs.make_links(L, "haar", inputs.rng_for(1221, 0))
    h = dsb.Handle(L)
    dsb.dsbcg_stage_links(h, dev(U))
    dsb.dsbcg_apply_A(h, dev(U2), KAPPA, dev(X))  # converts U2: the staged copy is gone
    with pytest.raises(dsb.DSBCGError):
        dsb.dsbcg_apply_A(h, None, KAPPA, dev(X))
    with pytest.raises(dsb.DSBCGError):
        dsb.dsbcg_apply_A(dsb.Handle(L), None, KAPPA, dev(X))  # never staged
    bad = U.copy()
    bad[3, 1, 0, 2] = np.nan
    with pytest.raises(dsb.NotHPDError):
        dsb.dsbcg_stage_links(h, dev(bad))
