"""ctypes access to the C oracle of the Wilson-Dirac operator (test infrastructure).

Fields are numpy complex128 arrays in the layouts
  U   (V, 4, 3, 3)   psi (V, 4, 3, m)
and L = (Lx, Ly, Lz, Lt) with x fastest.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def load():
    """Load liboracle.so, building it first only if it is not there."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "liboracle.so")
    if not os.path.exists(path):
        from .build import build
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.oracle_gamma.argtypes = [ctypes.c_int, P]
    lib.oracle_neighbors.argtypes = [P, P]
    lib.oracle_apply_D.argtypes = [P, P, dbl, P, P, i32, i32]
    lib.oracle_apply_A.argtypes = [P, P, dbl, P, P, i32]
    lib.oracle_apply_A.restype = ctypes.c_int
    lib.oracle_apply_D_sites.argtypes = [P, P, dbl, P, i32, i32, P, i64, P]
    lib.oracle_apply_A_sites.argtypes = [P, P, dbl, P, i32, P, i64, P]
    lib.oracle_apply_A_sites.restype = ctypes.c_int
    lib.oracle_link_grad.argtypes = [P, dbl, P, P, i32, P]
    lib.oracle_max_threads.restype = ctypes.c_int
    _LIB = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _L(L) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(L, dtype=np.int32))


def _field(a, V: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.shape[0] != V or a.shape[1:3] != (4, 3):
        raise ValueError(f"field shape {a.shape} does not match ({V}, 4, 3, m)")
    return a


def _links(U, V: int) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.complex128)
    if U.shape != (V, 4, 3, 3):
        raise ValueError(f"links shape {U.shape} != ({V}, 4, 3, 3)")
    return U


def _vol(L) -> int:
    return int(np.prod(np.asarray(L, dtype=np.int64)))


def gamma(mu: int) -> np.ndarray:
    out = np.empty(16, dtype=np.complex128)
    load().oracle_gamma(mu, _ptr(out))
    return out.reshape(4, 4)


def neighbors(L) -> np.ndarray:
    V = _vol(L)
    out = np.empty((V, 8), dtype=np.int32)
    Lc = _L(L)
    load().oracle_neighbors(_ptr(Lc), _ptr(out))
    return out


def _as4(psi):
    psi = np.asarray(psi)
    return psi[..., None] if psi.ndim == 3 else psi


def apply_D(L, U, kappa: float, psi, dagger: bool = False) -> np.ndarray:
    """D psi, or D^H psi when dagger is set; psi of shape (V, 4, 3, m) or (V, 4, 3)."""
    V = _vol(L)
    squeeze = np.asarray(psi).ndim == 3
    psi = _field(_as4(psi), V)
    U = _links(U, V)
    out = np.empty_like(psi)
    Lc = _L(L)
    load().oracle_apply_D(_ptr(Lc), _ptr(U), float(kappa), _ptr(psi), _ptr(out),
                          psi.shape[3], int(bool(dagger)))
    return out[..., 0] if squeeze else out


def apply_A(L, U, kappa: float, psi) -> np.ndarray:
    """A psi = D^H D psi."""
    V = _vol(L)
    squeeze = np.asarray(psi).ndim == 3
    psi = _field(_as4(psi), V)
    U = _links(U, V)
    out = np.empty_like(psi)
    Lc = _L(L)
    if load().oracle_apply_A(_ptr(Lc), _ptr(U), float(kappa), _ptr(psi), _ptr(out),
                             psi.shape[3]) != 0:
        raise MemoryError("oracle_apply_A: allocation failed")
    return out[..., 0] if squeeze else out


def apply_D_sites(L, U, kappa: float, psi, sites, dagger: bool = False) -> np.ndarray:
    """(D psi)(x) or (D^H psi)(x) at the listed sites; shape (len(sites), 4, 3, m)."""
    V = _vol(L)
    psi = _field(_as4(psi), V)
    U = _links(U, V)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), 4, 3, psi.shape[3]), dtype=np.complex128)
    Lc = _L(L)
    load().oracle_apply_D_sites(_ptr(Lc), _ptr(U), float(kappa), _ptr(psi), psi.shape[3],
                                int(bool(dagger)), _ptr(sites), len(sites), _ptr(out))
    return out


def apply_A_sites(L, U, kappa: float, psi, sites) -> np.ndarray:
    """(A psi)(x) at the listed sites; shape (len(sites), 4, 3, m)."""
    V = _vol(L)
    psi = _field(_as4(psi), V)
    U = _links(U, V)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), 4, 3, psi.shape[3]), dtype=np.complex128)
    Lc = _L(L)
    if load().oracle_apply_A_sites(_ptr(Lc), _ptr(U), float(kappa), _ptr(psi), psi.shape[3],
                                   _ptr(sites), len(sites), _ptr(out)) != 0:
        raise MemoryError("oracle_apply_A_sites: allocation failed")
    return out


def link_grad(L, kappa: float, phi, psi) -> np.ndarray:
    """d/dU of Re<phi, D psi> (summed over columns) as dRe + i dIm, shape (V, 4, 3, 3)."""
    V = _vol(L)
    phi = _field(_as4(phi), V)
    psi = _field(_as4(psi), V)
    if phi.shape != psi.shape:
        raise ValueError("phi and psi must have the same shape")
    out = np.empty((V, 4, 3, 3), dtype=np.complex128)
    Lc = _L(L)
    load().oracle_link_grad(_ptr(Lc), float(kappa), _ptr(phi), _ptr(psi), phi.shape[3],
                            _ptr(out))
    return out


def max_threads() -> int:
    return int(load().oracle_max_threads())
