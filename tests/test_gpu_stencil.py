"""HIP Wilson stencil against the CPU oracle: neighbour tables (bit-exact), D, D^H
and A = D^H D in FP64 (<= 1e-13) and FP32 (<= 1e-5), at small lattices that span
several workgroups with a ragged tail, and at the full workload sizes on sampled
sites."""
import numpy as np
import pytest

import oracle
from paper_1205_0359_amd import inputs
import paper_1205_0359_amd as dsb

from gpu_util import announce, dev, host, rel_max

pytestmark = pytest.mark.gpu

LATTICES = [(4, 4, 4, 4), (3, 4, 5, 6), (2, 2, 2, 2), (8, 6, 4, 10), (5, 3, 7, 2)]


@pytest.mark.parametrize("L", LATTICES)
def test_neighbour_table_bit_exact(L):
    announce("neighbors", L)
    h = dsb.Handle(L)
    assert np.array_equal(dsb.dsbcg_neighbors(h), oracle.neighbors(L))


def _case(L, m, seed, kind="haar"):
    U = inputs.make_links(L, kind, inputs.rng_for(seed, 0))
    X = inputs.gaussian_rhs(inputs.rng_for(seed, 1), int(np.prod(L)), m)
    return U, X


@pytest.mark.parametrize("L,m", [((4, 4, 4, 4), 1), ((4, 4, 4, 4), 4), ((3, 4, 5, 6), 5),
                                 ((4, 2, 6, 4), 12), ((2, 4, 4, 6), 16), ((8, 6, 4, 10), 7),
                                 ((5, 3, 7, 2), 3)])
def test_apply_A_fp64(L, m):
    announce("apply_A fp64", L, m)
    kappa = 0.124
    U, X = _case(L, m, 700 + m)
    h = dsb.Handle(L)
    Y = host(dsb.dsbcg_apply_A(h, dev(U), kappa, dev(X)))
    want = oracle.apply_A(L, U, kappa, X)
    assert rel_max(Y, want) <= 1e-13


@pytest.mark.parametrize("L,m", [((4, 4, 4, 4), 3), ((3, 4, 5, 6), 8), ((8, 6, 4, 10), 11),
                                 ((5, 3, 7, 2), 5), ((3, 4, 5, 6), 6), ((8, 6, 4, 10), 7)])
def test_apply_D_and_adjoint_fp64(L, m):
    announce("apply_D fp64", L, m)
    kappa = 0.13
    U, X = _case(L, m, 720 + m, "smooth")
    h = dsb.Handle(L)
    for dag in (False, True):
        Y = host(dsb.dsbcg_apply_D(h, dev(U), kappa, dev(X), dagger=dag))
        want = oracle.apply_D(L, U, kappa, X, dagger=dag)
        assert rel_max(Y, want) <= 1e-13


@pytest.mark.parametrize("L,m", [((4, 4, 4, 4), 4), ((3, 4, 5, 6), 5), ((8, 6, 4, 10), 12),
                                 ((2, 2, 2, 2), 1)])
def test_apply_A_fp32(L, m):
    announce("apply_A fp32", L, m)
    kappa = 0.12
    U, X = _case(L, m, 740 + m)
    h = dsb.Handle(L)
    Y = host(dsb.dsbcg_apply_A(h, dev(U), kappa, dev(X), precision=dsb.DSBCG_FP32_RELIABLE))
    want = oracle.apply_A(L, U, kappa, X)
    err = rel_max(Y, want)
    assert err <= 1e-5
    assert err > 1e-9  # really computed in single precision


def test_repeatable_bitwise():
    L, m = (8, 6, 4, 10), 6
    announce("apply_A repeat", L, m)
    U, X = _case(L, m, 760)
    h = dsb.Handle(L)
    dU, dX = dev(U), dev(X)
    a = host(dsb.dsbcg_apply_A(h, dU, 0.12, dX))
    b = host(dsb.dsbcg_apply_A(h, dU, 0.12, dX))
    assert np.array_equal(a, b)


def test_argument_errors():
    h = dsb.Handle((4, 4, 4, 4))
    U, X = _case((4, 4, 4, 4), 2, 770)
    dU, dX = dev(U), dev(X)
    with pytest.raises(dsb.DSBCGError):
        dsb.dsbcg_apply_A(h, dU, float("nan"), dX)
    with pytest.raises(dsb.DSBCGError):
        dsb.dsbcg_apply_A(h, dU, 0.1, dX, Y=dX)
    import torch
    big = torch.zeros((256, 4, 3, 17), dtype=torch.complex128, device="cuda")
    with pytest.raises(dsb.DSBCGError):
        dsb.dsbcg_apply_A(h, dU, 0.1, big)


@pytest.mark.parametrize("name", ["smooth16^4_m12_s8", "haar24^3x48_m12_s12",
                                  "haar32^3x64_m8r5_s10"])
def test_apply_A_full_size_sampled(name):
    """The workload's own shapes; the oracle evaluates A at 48 sampled sites."""
    w = inputs.WORKLOADS[name]
    announce("apply_A full size", name)
    U, B = w.make()
    h = dsb.Handle(w.L)
    rng = np.random.default_rng(5)
    sites = np.concatenate([[0, w.V - 1], rng.integers(0, w.V, 46)])
    dU, dB = dev(U), dev(B)
    for prec, bound in ((dsb.DSBCG_FP64, 1e-13), (dsb.DSBCG_FP32_RELIABLE, 1e-5)):
        Y = dsb.dsbcg_apply_A(h, dU, w.kappa, dB, precision=prec)
        import torch
        got = host(Y[torch.from_numpy(sites).to('cuda')])
        want = oracle.apply_A_sites(w.L, U, w.kappa, B, sites)
        assert rel_max(got, want) <= bound, prec
        del Y


def test_apply_A_full_size_five_columns():
    """32^3 x 64 with the five columns of the deflated block (the FP64 kernel
    that reads its links from global memory): the oracle evaluates A at 48
    sampled sites."""
    w = inputs.WORKLOADS["haar32^3x64_m8r5_s10"]
    announce("apply_A full size, 5 columns", w.name)
    U, B = w.make()
    B5 = np.ascontiguousarray(B[..., [0, 1, 3, 4, 6]])
    del B
    h = dsb.Handle(w.L)
    rng = np.random.default_rng(6)
    sites = np.concatenate([[0, w.V - 1], rng.integers(0, w.V, 46)])
    import torch
    Y = dsb.dsbcg_apply_A(h, dev(U), w.kappa, dev(B5))
    got = host(Y[torch.from_numpy(sites).to('cuda')])
    want = oracle.apply_A_sites(w.L, U, w.kappa, B5, sites)
    assert rel_max(got, want) <= 1e-13
