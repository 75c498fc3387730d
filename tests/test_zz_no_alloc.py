"""dsbcg_apply_A_noalloc, the entry point that allocates no device memory,
against dsbcg_apply_A (the same kernels in the same order: equal bit for bit,
and within the FP64 stencil tolerance 1e-13 of the oracle), through the C ABI:
two calls in a row on one GPU, the second with a smaller input (fewer
columns, a smaller lattice), in both precisions, with U passed and with the
staged links; and the size limit of the workspace."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1205_0359_amd import _lib, inputs
import paper_1205_0359_amd as dsb

from gpu_util import announce, dev, host, rel_max

pytestmark = pytest.mark.gpu

KAPPA = 0.124


def _noalloc():
    lib = _lib.load()
    f = lib.dsbcg_apply_A_noalloc
    P = ctypes.c_void_p
    f.argtypes = [P, P, ctypes.c_double, P, P, ctypes.c_int32, ctypes.c_int32, P]
    f.restype = ctypes.c_int
    return f


def _call(h, U, X, precision):
    import torch
    Y = torch.full_like(X, float("nan"))
    code = _noalloc()(h.ptr, None if U is None else ctypes.c_void_p(U.data_ptr()), KAPPA,
                      ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()), X.shape[-1], precision,
                      _lib._stream(None))
    _lib._check(code)
    return host(Y)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("staged", [False, True])
def test_noalloc_equals_apply_A_twice_second_smaller(precision, staged):
    for L, m, seed in (((6, 4, 6, 8), 7, 1300), ((4, 4, 4, 4), 3, 1301)):
        announce("noalloc", L, m, "precision", precision, "staged", staged)
        U = inputs.make_links(L, "haar", inputs.rng_for(seed, 0))
        X = inputs.gaussian_rhs(inputs.rng_for(seed, 1), int(np.prod(L)), m)
        h = dsb.Handle(L)
        dU, dX = dev(U), dev(X)
        want = host(dsb.dsbcg_apply_A(h, dU, KAPPA, dX, precision=precision))
        if staged:
            dsb.dsbcg_stage_links(h, dU)
        got = _call(h, None if staged else dU, dX, precision)
        assert np.array_equal(got, want)
        ref = oracle.apply_A(L, U, KAPPA, X)
        assert rel_max(got, ref) <= (1e-13 if precision == 0 else 1e-5)


def test_noalloc_rejects_inputs_beyond_the_workspace():
    L, m = (16, 16, 16, 16), 4  # 65536 sites: the links and 2 blocks of 12 V m complex128 exceed 128 MiB
    announce("noalloc limit", L, m)
    import torch
    h = dsb.Handle(L)
    U = torch.zeros((65536, 4, 3, 3), dtype=torch.complex128, device="cuda")
    X = torch.zeros((65536, 4, 3, m), dtype=torch.complex128, device="cuda")
    Y = torch.zeros_like(X)
    code = _noalloc()(h.ptr, ctypes.c_void_p(U.data_ptr()), KAPPA, ctypes.c_void_p(X.data_ptr()),
                      ctypes.c_void_p(Y.data_ptr()), m, 0, _lib._stream(None))
    assert code == _lib.DSBCG_ERR_ARG
    assert b"workspace" in _lib.load().dsbcg_last_error()
