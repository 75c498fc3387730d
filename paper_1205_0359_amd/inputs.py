"""Seeded synthetic inputs for the shifted multi-RHS Wilson systems.

This module only draws random numbers and lays them out; it holds none of the
solver's arithmetic, so both the HIP path and the CPU oracle take their inputs
from here.

Layouts (C order, complex128):
  links  U[V, 4, 3, 3]   U[x, mu] is the SU(3) matrix on the link x -> x+mu
  rhs    B[V, 4, 3, m]   site-major, spin, colour, right-hand side innermost
Site index: x + Lx*(y + Ly*(z + Lz*t)).

The paper's own workloads use a quenched gauge configuration and "random"
right-hand sides (Sec. 4); neither the configuration nor its generator is
available, so Haar-random or smooth random SU(3) fields stand in for it.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "rng_for", "complex_gaussian", "haar_su3",
    "smooth_su3", "unit_links", "gaussian_rhs", "z2_rhs", "deflating_rhs",
    "make_links", "make_rhs", "volume", "site_coordinates", "plane_wave",
]


def volume(L) -> int:
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def rng_for(workload_id: int, stream: int) -> np.random.Generator:
    """Generator for one input stream of one workload.

    stream 0: links, 1: right-hand sides, 2: noise / loss weights, 3: picks.
    """
    return np.random.Generator(np.random.PCG64(1000 * workload_id + stream))


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """Entries with independent real and imaginary parts ~ N(0, 1/2)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    out = np.empty(shape, dtype=np.complex128)
    out.real = re
    out.imag = im
    out *= np.sqrt(0.5)
    return out


def _orthonormal_columns(Z: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on the columns of a stack of 3x3 matrices.

    Equals Q diag(R_ii/|R_ii|) of a QR factorisation (the unique QR with a
    positive real R diagonal), which makes Q Haar-distributed on U(3) when Z
    is complex Gaussian.
    """
    Q = _gram_schmidt3(Z)
    # a second pass removes the rounding left by the first; its R factor is
    # upper triangular with a positive diagonal, so Q is unchanged in exact
    # arithmetic
    return _gram_schmidt3(Q)


def _gram_schmidt3(Z: np.ndarray) -> np.ndarray:
    Q = np.empty_like(Z)
    q0 = Z[..., :, 0]
    q0 = q0 / np.linalg.norm(q0, axis=-1, keepdims=True)
    q1 = Z[..., :, 1]
    q1 = q1 - q0 * np.sum(q0.conj() * q1, axis=-1, keepdims=True)
    q1 = q1 / np.linalg.norm(q1, axis=-1, keepdims=True)
    q2 = Z[..., :, 2]
    q2 = q2 - q0 * np.sum(q0.conj() * q2, axis=-1, keepdims=True)
    q2 = q2 - q1 * np.sum(q1.conj() * q2, axis=-1, keepdims=True)
    q2 = q2 / np.linalg.norm(q2, axis=-1, keepdims=True)
    Q[..., :, 0] = q0
    Q[..., :, 1] = q1
    Q[..., :, 2] = q2
    return Q


def _det3(U: np.ndarray) -> np.ndarray:
    return (U[..., 0, 0] * (U[..., 1, 1] * U[..., 2, 2] - U[..., 1, 2] * U[..., 2, 1])
            - U[..., 0, 1] * (U[..., 1, 0] * U[..., 2, 2] - U[..., 1, 2] * U[..., 2, 0])
            + U[..., 0, 2] * (U[..., 1, 0] * U[..., 2, 1] - U[..., 1, 1] * U[..., 2, 0]))


def haar_su3(rng: np.random.Generator, count: int, chunk: int = 1 << 20) -> np.ndarray:
    """`count` Haar-random SU(3) matrices, shape (count, 3, 3).

    Haar on U(3) from the phase-fixed QR of a complex Gaussian matrix, then
    division by the principal cube root of the determinant; left invariance
    of the U(3) measure carries over, so the result is Haar on SU(3).
    """
    out = np.empty((count, 3, 3), dtype=np.complex128)
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        Q = _orthonormal_columns(complex_gaussian(rng, (e - s, 3, 3)))
        d = _det3(Q)
        Q /= np.exp(1j * np.angle(d) / 3.0)[:, None, None]
        out[s:e] = Q
    return out


def smooth_su3(rng: np.random.Generator, count: int, eps: float,
               chunk: int = 1 << 20) -> np.ndarray:
    """SU(3) matrices exp(i*eps*H) with H random traceless Hermitian.

    H = (G + G^H)/2 - tr/3 * I with complex Gaussian G (entries N(0,1),
    real and imaginary parts each N(0, 1/2)); the exponential is taken through
    the eigendecomposition of H, so det = exp(i*eps*tr H) = 1.
    """
    out = np.empty((count, 3, 3), dtype=np.complex128)
    eye = np.eye(3)
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        G = complex_gaussian(rng, (e - s, 3, 3))
        H = 0.5 * (G + np.conj(np.swapaxes(G, -1, -2)))
        tr = np.trace(H, axis1=-2, axis2=-1).real
        H = H - (tr / 3.0)[:, None, None] * eye
        w, Q = np.linalg.eigh(H)
        ph = np.exp(1j * eps * w)
        out[s:e] = (Q * ph[:, None, :]) @ np.conj(np.swapaxes(Q, -1, -2))
    return out


def unit_links(L) -> np.ndarray:
    V = volume(L)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def make_links(L, kind: str, rng: np.random.Generator, eps: float = 0.3) -> np.ndarray:
    V = volume(L)
    if kind == "haar":
        return haar_su3(rng, 4 * V).reshape(V, 4, 3, 3)
    if kind == "smooth":
        return smooth_su3(rng, 4 * V, eps).reshape(V, 4, 3, 3)
    if kind == "unit":
        return unit_links(L)
    raise ValueError(f"unknown link kind {kind!r}")


def gaussian_rhs(rng: np.random.Generator, V: int, m: int) -> np.ndarray:
    return complex_gaussian(rng, (V, 4, 3, m))


def z2_rhs(rng: np.random.Generator, V: int, m: int) -> np.ndarray:
    """(+-1 +- i)/sqrt(2) with independent signs for real and imaginary parts."""
    re = rng.integers(0, 2, size=(V, 4, 3, m)) * 2 - 1
    im = rng.integers(0, 2, size=(V, 4, 3, m)) * 2 - 1
    return (re + 1j * im) / np.sqrt(2.0)


def deflating_rhs(rng: np.random.Generator, noise_rng: np.random.Generator, V: int) -> np.ndarray:
    """Eight right-hand sides of rank five.

    Columns 0, 1, 3, 4, 6 are complex Gaussian; column 2 repeats column 0,
    column 5 repeats column 1 and column 7 is column 4 plus 1e-12 Gaussian
    noise.
    """
    B = np.empty((V, 4, 3, 8), dtype=np.complex128)
    for col in (0, 1, 3, 4, 6):
        B[..., col] = complex_gaussian(rng, (V, 4, 3))
    B[..., 2] = B[..., 0]
    B[..., 5] = B[..., 1]
    B[..., 7] = B[..., 4] + 1e-12 * complex_gaussian(noise_rng, (V, 4, 3))
    return B


def site_coordinates(L) -> np.ndarray:
    """(V, 4) integer coordinates (x, y, z, t) of site x + Lx (y + Ly (z + Lz t))."""
    V = volume(L)
    idx = np.arange(V)
    out = np.empty((V, 4), dtype=np.int64)
    for d in range(4):
        out[:, d] = idx % L[d]
        idx = idx // L[d]
    return out


def plane_wave(L, nvec, chi: np.ndarray) -> np.ndarray:
    """(V, 4, 3) field exp(i p.x) chi with p_mu = 2 pi nvec_mu / L_mu and chi a
    (4, 3) spin-colour vector."""
    p = 2.0 * np.pi * np.asarray(nvec, dtype=np.float64) / np.asarray(L, dtype=np.float64)
    phase = np.exp(1j * (site_coordinates(L) @ p))
    return phase[:, None, None] * np.asarray(chi, dtype=np.complex128)[None]


def make_rhs(kind: str, V: int, m: int, rng: np.random.Generator,
             noise_rng: np.random.Generator | None = None) -> np.ndarray:
    if kind == "gaussian":
        return gaussian_rhs(rng, V, m)
    if kind == "z2":
        return z2_rhs(rng, V, m)
    if kind == "deflating":
        if m != 8:
            raise ValueError("the deflating right-hand sides have m = 8")
        return deflating_rhs(rng, noise_rng, V)
    raise ValueError(f"unknown rhs kind {kind!r}")


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic problem: lattice, links, kappa, right-hand sides, shifts."""
    wid: int
    name: str
    L: tuple
    kappa: float
    links: str
    rhs: str
    m: int
    shifts: tuple
    tol: float
    eps: float = 0.3

    @property
    def V(self) -> int:
        return volume(self.L)

    @property
    def n(self) -> int:
        return 12 * self.V

    def make(self, links: bool = True, rhs: bool = True):
        U = make_links(self.L, self.links, rng_for(self.wid, 0), self.eps) if links else None
        B = (make_rhs(self.rhs, self.V, self.m, rng_for(self.wid, 1), rng_for(self.wid, 2))
             if rhs else None)
        return U, B


def _logspace(lo, hi, k):
    return tuple(float(v) for v in np.logspace(lo, hi, k))


WORKLOADS = {
    # 4^4, Haar links: small enough for the dense Cholesky cross-check.
    "haar4^4_m4_s3": Workload(1, "haar4^4_m4_s3", (4, 4, 4, 4), 0.12, "haar", "gaussian", 4,
                             (1e-3, 1e-2, 1e-1), 1e-10),
    # 16^4, smooth links exp(0.3 i H), Z2 noise, eight shifts in [1e-4, 1].
    "smooth16^4_m12_s8": Workload(2, "smooth16^4_m12_s8", (16, 16, 16, 16), 0.125, "smooth", "z2",
                                  12, _logspace(-4, 0, 8), 1e-10),
    # 24^3 x 48, Haar links, twelve shifts in [1e-5, 1].
    "haar24^3x48_m12_s12": Workload(3, "haar24^3x48_m12_s12", (24, 24, 24, 48), 0.12, "haar",
                                    "gaussian", 12, _logspace(-5, 0, 12), 1e-10),
    # differentiation workload (16^4 timing size; the FD check runs at 4^4).
    "smooth16^4_m4_s6_grad": Workload(4, "smooth16^4_m4_s6_grad", (16, 16, 16, 16), 0.125,
                                      "smooth", "gaussian", 4, _logspace(-3, 0, 6), 1e-10),
    # 32^3 x 64, Haar links, eight right-hand sides of rank five, ten shifts.
    "haar32^3x64_m8r5_s10": Workload(5, "haar32^3x64_m8r5_s10", (32, 32, 32, 64), 0.124, "haar",
                                     "deflating", 8, _logspace(-5, 0, 10), 1e-10),
}
