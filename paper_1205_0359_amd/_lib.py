"""Thin ctypes binding of libdsbcg.so (the C ABI in include/dsbcg.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory and the stream.  There is no CPU
fallback; if the library is missing the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsbcg.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "dsbcg.h")

DSBCG_OK = 0
DSBCG_ERR_ARG = 1
DSBCG_ERR_NOT_HPD = 2
DSBCG_ERR_NOT_CONVERGED = 3
DSBCG_ERR_HIP = 4
DSBCG_ERR_OOM = 5
DSBCG_FP64 = 0
DSBCG_FP32_RELIABLE = 1
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_NOT_HPD", 3: "ERR_NOT_CONVERGED", 4: "ERR_HIP",
                5: "ERR_OOM"}


class DSBCGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class NotHPDError(DSBCGError):
    pass


class NotConvergedError(DSBCGError):
    pass


class dsbcg_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("fixed_iters", ctypes.c_int32), ("ru_interval", ctypes.c_int32),
                ("tau_B", ctypes.c_double),
                ("tau_W", ctypes.c_double), ("refine", ctypes.c_int32),
                ("freeze", ctypes.c_int32), ("window", ctypes.c_int32),
                ("switch_at", ctypes.c_double), ("keep_workspace", ctypes.c_int32),
                ("vector_stop", ctypes.c_int32)]


class dsbcg_stats(ctypes.Structure):
    _fields_ = [("block_iters", ctypes.c_int32), ("rank0", ctypes.c_int32),
                ("deflations", ctypes.c_int32), ("reliable_updates", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("final_width", ctypes.c_int32),
                ("switch_iter", ctypes.c_int32), ("qr2_skipped", ctypes.c_int32),
                ("main_relres_max", ctypes.c_double),
                ("mvms", ctypes.c_int64),
                ("est_relres", ctypes.POINTER(ctypes.c_double)),
                ("true_relres", ctypes.POINTER(ctypes.c_double)),
                ("widths", ctypes.POINTER(ctypes.c_int32)), ("widths_len", ctypes.c_int32),
                ("qr_redone", ctypes.c_int32), ("mvms_vector", ctypes.c_int64),
                ("frozen_at", ctypes.POINTER(ctypes.c_int32)),
                ("est_history", ctypes.POINTER(ctypes.c_double))]


_lib = None


def load():
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1205_0359_amd/build.py "
                           "(there is no CPU fallback)")
    # PyTorch ships its own HIP runtime (same soname as the system one).  Load
    # it first so that the library binds to that copy: two HIP runtimes in one
    # process cannot share the device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.dsbcg_default_opts.argtypes = [ctypes.POINTER(dsbcg_opts)]
    lib.dsbcg_default_opts.restype = None
    lib.dsbcg_create.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(P)]
    lib.dsbcg_create.restype = ctypes.c_int
    lib.dsbcg_destroy.argtypes = [P]
    lib.dsbcg_destroy.restype = None
    lib.dsbcg_neighbors.argtypes = [P, P]
    lib.dsbcg_neighbors.restype = ctypes.c_int
    lib.dsbcg_apply_A.argtypes = [P, P, dbl, P, P, i32, i32, P]
    lib.dsbcg_apply_A.restype = ctypes.c_int
    lib.dsbcg_release_workspace.argtypes = [P]
    lib.dsbcg_release_workspace.restype = ctypes.c_int
    lib.dsbcg_stage_links.argtypes = [P, P, P]
    lib.dsbcg_stage_links.restype = ctypes.c_int
    lib.dsbcg_apply_A_noalloc.argtypes = [P, P, dbl, P, P, i32, i32, P]
    lib.dsbcg_apply_A_noalloc.restype = ctypes.c_int
    lib.dsbcg_apply_D.argtypes = [P, P, dbl, P, P, i32, i32, P]
    lib.dsbcg_apply_D.restype = ctypes.c_int
    lib.dsbcg_solve.argtypes = [P, P, dbl, P, i32, ctypes.POINTER(ctypes.c_double), i32, dbl,
                                ctypes.POINTER(dsbcg_opts), P, ctypes.POINTER(dsbcg_stats), P]
    lib.dsbcg_solve.restype = ctypes.c_int
    lib.dsbcg_solve_multi.argtypes = lib.dsbcg_solve.argtypes
    lib.dsbcg_solve_multi.restype = ctypes.c_int
    lib.dsbcg_solve_rational.argtypes = [P, P, dbl, P, i32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double), i32, dbl, dbl,
                                         ctypes.POINTER(dsbcg_opts), P, ctypes.POINTER(dsbcg_stats), P]
    lib.dsbcg_solve_rational.restype = ctypes.c_int
    lib.dsbcg_grad.argtypes = [P, P, dbl, ctypes.POINTER(ctypes.c_double), i32, i32, P, P, P, P,
                               ctypes.POINTER(ctypes.c_double), P]
    lib.dsbcg_grad.restype = ctypes.c_int
    lib.dsbcg_link_grad.argtypes = [P, dbl, P, P, i32, P, P]
    lib.dsbcg_link_grad.restype = ctypes.c_int
    lib.dsbcg_profile_enable.argtypes = [P, i32]
    lib.dsbcg_profile_enable.restype = ctypes.c_int
    lib.dsbcg_profile_read.argtypes = [P, i32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    lib.dsbcg_profile_read.restype = ctypes.c_int
    lib.dsbcg_profile_select.argtypes = [P, ctypes.c_uint32]
    lib.dsbcg_profile_select.restype = ctypes.c_int
    lib.dsbcg_profile_name.argtypes = [i32]
    lib.dsbcg_profile_name.restype = ctypes.c_char_p
    lib.dsbcg_last_error.argtypes = []
    lib.dsbcg_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def header_functions() -> list[str]:
    """Names of the functions declared in include/dsbcg.h."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dsbcg_[a-z_A-Z0-9]+)\s*\(", txt)))


def _check(code: int):
    if code == DSBCG_OK:
        return
    msg = load().dsbcg_last_error().decode(errors="replace")
    if code == DSBCG_ERR_NOT_HPD:
        raise NotHPDError(code, msg)
    if code == DSBCG_ERR_NOT_CONVERGED:
        raise NotConvergedError(code, msg)
    raise DSBCGError(code, msg)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the DSBlockCG library needs a HIP device (there is no CPU fallback)")
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _links(U, h):
    """Pointer to U, or NULL (the handle's staged links) when U is None."""
    if U is None:
        return None
    return _dev(U, "U", (h.V, 4, 3, 3))


def _dev(t, name, shape=None, dtype=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if dtype is None:
        dtype = torch.complex128
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Handle:
    """A dsbcg_handle bound to one lattice (owns its neighbour geometry and workspace)."""

    def __init__(self, L):
        lib = load()
        self.L = tuple(int(v) for v in L)
        self.V = self.L[0] * self.L[1] * self.L[2] * self.L[3]
        arr = (ctypes.c_int32 * 4)(*self.L)
        h = ctypes.c_void_p()
        _check(lib.dsbcg_create(arr, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().dsbcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ptr(self):
        if not self._h:
            raise RuntimeError("handle is closed")
        return self._h


def dsbcg_neighbors(h: Handle):
    import numpy as np
    out = np.empty((h.V, 8), dtype=np.int32)
    _check(load().dsbcg_neighbors(h.ptr, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def dsbcg_release_workspace(h: Handle):
    """Free the device workspace the handle holds (the staged links stay)."""
    _check(load().dsbcg_release_workspace(h.ptr))


def dsbcg_stage_links(h: Handle, U, stream=None):
    """Check and convert U once; later calls may pass U=None to use this copy."""
    _check(load().dsbcg_stage_links(h.ptr, _dev(U, "U", (h.V, 4, 3, 3)), _stream(stream)))


def dsbcg_apply_A(h: Handle, U, kappa: float, X, Y=None, precision: int = DSBCG_FP64,
                  stream=None):
    """Y = A X = D^H D X; X, Y complex128 (V, 4, 3, m) device tensors."""
    torch = _torch()
    m = X.shape[-1]
    pU = _links(U, h)
    pX = _dev(X, "X", (h.V, 4, 3, m))
    if Y is None:
        Y = torch.empty_like(X)
    pY = _dev(Y, "Y", (h.V, 4, 3, m))
    _check(load().dsbcg_apply_A(h.ptr, pU, float(kappa), pX, pY, int(m), int(precision),
                                _stream(stream)))
    return Y


def dsbcg_apply_A_noalloc(h: Handle, U, kappa: float, X, Y, precision: int = DSBCG_FP64,
                          stream=None):
    """Y = A X into the caller's Y with no device allocation by the library."""
    m = X.shape[-1]
    pX = _dev(X, "X", (h.V, 4, 3, m))
    pY = _dev(Y, "Y", (h.V, 4, 3, m))
    _check(load().dsbcg_apply_A_noalloc(h.ptr, _links(U, h), float(kappa), pX, pY, int(m), int(precision),
                                        _stream(stream)))
    return Y


def dsbcg_apply_D(h: Handle, U, kappa: float, X, Y=None, dagger: bool = False, stream=None):
    """Y = D X (or D^H X); FP64."""
    torch = _torch()
    m = X.shape[-1]
    pU = _links(U, h)
    pX = _dev(X, "X", (h.V, 4, 3, m))
    if Y is None:
        Y = torch.empty_like(X)
    pY = _dev(Y, "Y", (h.V, 4, 3, m))
    _check(load().dsbcg_apply_D(h.ptr, pU, float(kappa), pX, pY, int(m), int(bool(dagger)),
                                _stream(stream)))
    return Y


def default_opts(**kw) -> dsbcg_opts:
    o = dsbcg_opts()
    load().dsbcg_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k!r}")
        setattr(o, k, v)
    return o


_MAX_WIDTHS = 4096  # main-phase block widths reported per solve


def _new_stats(s, m):
    import numpy as np
    est = np.zeros(s * m)
    true = np.zeros(s * m)
    widths = np.zeros(_MAX_WIDTHS, dtype=np.int32)
    st = dsbcg_stats()
    st.est_relres = est.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st.true_relres = true.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st.widths = widths.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    st.widths_len = _MAX_WIDTHS
    frozen = np.zeros(s * m, dtype=np.int32)
    st.frozen_at = frozen.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    st._widths_buf = widths  # kept alive with the struct
    st._frozen_buf = frozen
    hist = np.zeros(_MAX_WIDTHS)
    st.est_history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st._hist_buf = hist
    return st, est, true


def _stats_dict(code, st, est, true, s, m):
    widths = st._widths_buf[:min(st.block_iters, _MAX_WIDTHS)].tolist()
    return {
        "widths": widths, "qr_redone": st.qr_redone,
        "status": STATUS_NAMES.get(code, code),
        "block_iters": st.block_iters, "rank0": st.rank0, "deflations": st.deflations,
        "reliable_updates": st.reliable_updates, "refine_iters": st.refine_iters,
        "final_width": st.final_width, "switch_iter": st.switch_iter, "qr2_skipped": st.qr2_skipped,
        "main_relres_max": st.main_relres_max, "mvms": int(st.mvms),
        "mvms_vector": int(st.mvms_vector), "frozen_at": st._frozen_buf.reshape(s, m).T.copy(),
        "est_history": st._hist_buf[:min(st.block_iters, _MAX_WIDTHS)].tolist(),
        "est_relres": est.reshape(s, m).T.copy(), "true_relres": true.reshape(s, m).T.copy(),
    }


def _solve(fn, h: Handle, U, kappa, B, sigma, tol, X, stream, raise_not_converged, multi, opts):
    import numpy as np
    torch = _torch()
    m = B.shape[-1]
    sig = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64).reshape(-1))
    s = len(sig)
    pU = _links(U, h)
    pB = _dev(B, "B", (s, h.V, 4, 3, m) if multi else (h.V, 4, 3, m))
    if X is None:
        X = torch.empty((s, h.V, 4, 3, m), dtype=torch.complex128, device=B.device)
    pX = _dev(X, "X", (s, h.V, 4, 3, m))
    o = default_opts(**opts)
    st, est, true = _new_stats(s, m)
    code = fn(h.ptr, pU, float(kappa), pB, int(m), sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
              int(s), float(tol), ctypes.byref(o), pX, ctypes.byref(st), _stream(stream))
    stats = _stats_dict(code, st, est, true, s, m)
    if code == DSBCG_ERR_NOT_CONVERGED and not raise_not_converged:
        return X, stats
    _check(code)
    return X, stats


def dsbcg_solve(h: Handle, U, kappa: float, B, sigma, tol: float, X=None, stream=None,
                raise_not_converged: bool = True, **opts):
    """Solve (sigma_j I + A) X_j = B for all shifts.

    Returns (X, stats) with X complex128 (s, V, 4, 3, m) on the device and a
    stats dict (iterations, mvms, estimated and true relative residuals as
    (m, s) arrays).
    """
    return _solve(load().dsbcg_solve, h, U, kappa, B, sigma, tol, X, stream, raise_not_converged,
                  False, opts)


def dsbcg_solve_multi(h: Handle, U, kappa: float, B, sigma, tol: float, X=None, stream=None,
                      raise_not_converged: bool = True, **opts):
    """Solve (sigma_j I + A) X_j = B_j with one block per shift, B of shape (s, V, 4, 3, m)."""
    return _solve(load().dsbcg_solve_multi, h, U, kappa, B, sigma, tol, X, stream,
                  raise_not_converged, True, opts)


def dsbcg_solve_rational(h: Handle, U, kappa: float, B, sigma, coef, c0: float, tol: float, Y=None,
                         stream=None, raise_not_converged: bool = True, **opts):
    """Partial-fraction sum Y = c0 B + sum_j coef_j (sigma_j I + A)^{-1} B.

    Returns (Y, stats) with Y complex128 (V, 4, 3, m) on the device.  In the
    FP64 form the per-shift solutions are never formed and stats
    "true_relres" holds -1 (not computed).
    """
    import numpy as np
    torch = _torch()
    m = B.shape[-1]
    sig = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64).reshape(-1))
    cf = np.ascontiguousarray(np.asarray(coef, dtype=np.float64).reshape(-1))
    s = len(sig)
    if len(cf) != s:
        raise ValueError("coef and sigma differ in length")
    pU = _links(U, h)
    pB = _dev(B, "B", (h.V, 4, 3, m))
    if Y is None:
        Y = torch.empty((h.V, 4, 3, m), dtype=torch.complex128, device=B.device)
    pY = _dev(Y, "Y", (h.V, 4, 3, m))
    o = default_opts(**opts)
    st, est, true = _new_stats(s, m)
    code = load().dsbcg_solve_rational(
        h.ptr, pU, float(kappa), pB, int(m), sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        cf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(s), float(c0), float(tol),
        ctypes.byref(o), pY, ctypes.byref(st), _stream(stream))
    stats = _stats_dict(code, st, est, true, s, m)
    if code == DSBCG_ERR_NOT_CONVERGED and not raise_not_converged:
        return Y, stats
    _check(code)
    return Y, stats


def dsbcg_grad(h: Handle, U, kappa: float, sigma, X, Lam, want_U=True, want_B=True,
               want_sigma=True, stream=None):
    """Backward kernels: (dU, dB, dsigma) from X_j and Lambda_j = (sigma_j + A)^{-1} G_j."""
    import numpy as np
    torch = _torch()
    s, V, _, _, m = X.shape
    sig = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64).reshape(-1))
    pU = _links(U, h)
    pX = _dev(X, "X", (s, h.V, 4, 3, m))
    pL = _dev(Lam, "Lam", (s, h.V, 4, 3, m))
    dU = torch.empty((h.V, 4, 3, 3), dtype=torch.complex128, device=X.device) if want_U else None
    dB = torch.empty((h.V, 4, 3, m), dtype=torch.complex128, device=X.device) if want_B else None
    ds = np.zeros(s) if want_sigma else None
    _check(load().dsbcg_grad(h.ptr, pU, float(kappa), sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             int(s), int(m), pX, pL,
                             ctypes.c_void_p(dU.data_ptr()) if dU is not None else None,
                             ctypes.c_void_p(dB.data_ptr()) if dB is not None else None,
                             ds.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if ds is not None else None,
                             _stream(stream)))
    return dU, dB, ds


def dsbcg_link_grad(h: Handle, kappa: float, Phi, Psi, dU=None, stream=None):
    """dU = d/dU sum_k Re <Phi_k, D[U] Psi_k> (dRe + i dIm); Phi, Psi (V, 4, 3, nvec)."""
    torch = _torch()
    nvec = Phi.shape[-1]
    pPhi = _dev(Phi, "Phi", (h.V, 4, 3, nvec))
    pPsi = _dev(Psi, "Psi", (h.V, 4, 3, nvec))
    if dU is None:
        dU = torch.empty((h.V, 4, 3, 3), dtype=torch.complex128, device=Phi.device)
    pdU = _dev(dU, "dU", (h.V, 4, 3, 3))
    _check(load().dsbcg_link_grad(h.ptr, float(kappa), pPhi, pPsi, int(nvec), pdU,
                                  _stream(stream)))
    return dU


def dsbcg_profile_enable(h: Handle, enable: bool = True):
    """Start (and reset) or stop per-kernel-class timing with HIP events."""
    _check(load().dsbcg_profile_enable(h.ptr, int(bool(enable))))


def dsbcg_profile_select(h: Handle, class_mask: int = 0xFFFFFFFF):
    """Time only the kernel classes whose bit is set (default: every class)."""
    _check(load().dsbcg_profile_select(h.ptr, int(class_mask) & 0xFFFFFFFF))


def dsbcg_profile_read(h: Handle) -> dict:
    """{class name: {"ms": total, "launches": n, "bytes": algorithmic bytes}}."""
    lib = load()
    out = {}
    k = 0
    while True:
        name = lib.dsbcg_profile_name(k)
        if not name:
            break
        ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(lib.dsbcg_profile_read(h.ptr, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
        out[name.decode()] = {"ms": ms.value, "launches": int(n.value), "bytes": by.value}
        k += 1
    return out
