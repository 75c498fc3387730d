"""Seeded synthetic inputs: SU(3) links and right-hand-side distributions."""
import numpy as np
import pytest

from paper_1205_0359_amd import inputs


def _unitarity_err(U):
    eye = np.eye(3)
    return np.abs(np.conj(np.swapaxes(U, -1, -2)) @ U - eye).max()


def test_haar_su3_is_special_unitary():
    U = inputs.haar_su3(inputs.rng_for(0, 0), 2000)
    assert _unitarity_err(U) < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


def test_haar_moments():
    # Haar on SU(3): E[tr U] = 0, E|tr U|^2 = 1, E|U_00|^2 = 1/3.
    U = inputs.haar_su3(inputs.rng_for(0, 1), 100_000)
    tr = np.trace(U, axis1=-2, axis2=-1)
    assert abs(tr.mean()) < 0.02
    assert abs(np.mean(np.abs(tr) ** 2) - 1.0) < 0.03
    assert abs(np.mean(np.abs(U[:, 0, 0]) ** 2) - 1.0 / 3.0) < 0.005


def test_smooth_su3():
    eps = 0.3
    U = inputs.smooth_su3(inputs.rng_for(0, 2), 2000, eps)
    assert _unitarity_err(U) < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
    # exp(i eps H) stays within ~eps*||H|| of the identity; Haar links do not
    dist = np.linalg.norm(U - np.eye(3), axis=(-2, -1)).mean()
    assert 0.1 < dist < 1.5


def test_rhs_distributions():
    V = 64
    B = inputs.gaussian_rhs(inputs.rng_for(0, 3), V, 5)
    assert B.shape == (V, 4, 3, 5)
    assert abs(np.mean(np.abs(B) ** 2) - 1.0) < 0.1
    Z = inputs.z2_rhs(inputs.rng_for(0, 4), V, 3)
    assert np.allclose(np.abs(Z.real), 1 / np.sqrt(2)) and np.allclose(np.abs(Z.imag), 1 / np.sqrt(2))
    # both signs occur independently in real and imaginary parts
    assert {(np.sign(z.real), np.sign(z.imag)) for z in Z.ravel()[:200]} == {
        (1, 1), (1, -1), (-1, 1), (-1, -1)}


def test_deflating_rhs_structure():
    V = 32
    B = inputs.deflating_rhs(inputs.rng_for(0, 5), inputs.rng_for(0, 6), V)
    assert np.array_equal(B[..., 2], B[..., 0])
    assert np.array_equal(B[..., 5], B[..., 1])
    d = np.linalg.norm(B[..., 7] - B[..., 4]) / np.linalg.norm(B[..., 4])
    assert 1e-13 < d < 1e-11
    s = np.linalg.svd(B.reshape(-1, 8), compute_uv=False)
    assert s[4] / s[0] > 0.1 and s[5] / s[0] < 1e-11


def test_seeded_and_reproducible():
    w = inputs.WORKLOADS["haar4^4_m4_s3"]
    U1, B1 = w.make()
    U2, B2 = w.make()
    assert np.array_equal(U1, U2) and np.array_equal(B1, B2)
    assert U1.shape == (256, 4, 3, 3) and B1.shape == (256, 4, 3, 4)


@pytest.mark.parametrize("name", list(inputs.WORKLOADS))
def test_workload_table(name):
    w = inputs.WORKLOADS[name]
    assert w.V == np.prod(w.L) and w.m >= 1 and len(w.shifts) >= 1
    assert all(sg > 0 for sg in w.shifts) and w.tol == 1e-10
