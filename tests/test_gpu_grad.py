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
