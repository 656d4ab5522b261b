"""Direct-sum oracle for the discrete FIO (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The product path never touches it.

Two independent implementations of eq:dfio (Sec. 1),

    u(x) = sum_{k in Omega} exp(2 pi i Phi(x,k)) f(k),  x in X,

and of its adjoint f(k) = sum_x exp(-2 pi i Phi(x,k)) u(x):

* ``forward`` / ``adjoint``: the C/OpenMP loop in ``direct.c`` (FP64), loaded
  through ctypes from ``liborc_direct.so`` (built by ``oracle/build.py``);
* ``forward_np`` / ``adjoint_np``: a numpy twin, vectorised over k, written
  separately so the two can be checked against each other.

The phase is evaluated in Cartesian k from its definition (eq:ex1, Sec. 5,
with the generalisation c_j -> a_j (2 + (1+eta_j) m_j(x)) / 3 used for the
learnable / perturbed variants).  The relative error metric of eq:err
(Sec. 5) is ``rel_err``.

Grid conventions: f has shape (N, N) with f[k1+N/2, k2+N/2]; u has shape
(N, N) with u[i1, i2] = u(i1/N, i2/N).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = os.path.join(_HERE, "liborc_direct.so")

FOURIER = 0
ELLIPSE = 1


@dataclass(frozen=True)
class Phase:
    """Phase descriptor.  kind FOURIER: Phi = x.k.  kind ELLIPSE: eq:ex1
    with c1 -> a1 (2 + (1+eta1) sin2pi x1 sin2pi x2)/3 and
    c2 -> a2 (2 + (1+eta2) cos2pi x1 cos2pi x2)/3."""

    kind: int = ELLIPSE
    a1: float = 1.0
    a2: float = 1.0
    eta1: float = 0.0
    eta2: float = 0.0


class _CPhase(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("a1", ctypes.c_double),
        ("a2", ctypes.c_double),
        ("eta1", ctypes.c_double),
        ("eta2", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBNAME):
            raise RuntimeError(
                f"{_LIBNAME} is missing; run oracle/build.py (or __graft_entry__.build())"
            )
        lib = ctypes.CDLL(_LIBNAME)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_direct_forward.argtypes = [
            ctypes.c_int, ctypes.POINTER(_CPhase), dp, ctypes.c_int, i64p, dp]
        lib.orc_direct_adjoint.argtypes = [
            ctypes.c_int, ctypes.POINTER(_CPhase), dp, ctypes.c_int, i64p, dp]
        lib.orc_phi.argtypes = [ctypes.POINTER(_CPhase)] + [ctypes.c_double] * 4
        lib.orc_phi.restype = ctypes.c_double
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _cphase(ph: Phase) -> _CPhase:
    return _CPhase(int(ph.kind), float(ph.a1), float(ph.a2), float(ph.eta1), float(ph.eta2))


def num_threads() -> int:
    """OpenMP threads the C oracle runs with."""
    return int(_load().orc_num_threads())


def phi_c(ph: Phase, x1: float, x2: float, k1: float, k2: float) -> float:
    """Phi(x,k) as evaluated by the C oracle (for unit tests of the phase)."""
    return float(_load().orc_phi(ctypes.byref(_cphase(ph)), x1, x2, k1, k2))


def forward(N: int, ph: Phase, f: np.ndarray, rows=None) -> np.ndarray:
    """u at ``rows`` (flat i1*N+i2; default: all of X) by the C direct sum."""
    lib = _load()
    f = np.ascontiguousarray(np.asarray(f, dtype=np.complex128).reshape(N, N))
    rows = np.arange(N * N, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.shape[0], dtype=np.complex128)
    lib.orc_direct_forward(
        N, ctypes.byref(_cphase(ph)),
        f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        int(rows.shape[0]), rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def adjoint(N: int, ph: Phase, u: np.ndarray, cols=None) -> np.ndarray:
    """f(k) = sum_x conj(exp(2 pi i Phi(x,k))) u(x) at ``cols`` (flat
    (k1+N/2)*N + (k2+N/2); default: all of Omega) by the C direct sum."""
    lib = _load()
    u = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(N, N))
    cols = np.arange(N * N, dtype=np.int64) if cols is None else np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros(cols.shape[0], dtype=np.complex128)
    lib.orc_direct_adjoint(
        N, ctypes.byref(_cphase(ph)),
        u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        int(cols.shape[0]), cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


# ----------------------------------------------------------------------------
# numpy twin (independent code, same definition)
# ----------------------------------------------------------------------------

def phi_np(ph: Phase, x1, x2, k1, k2):
    """Phi(x,k) by numpy broadcasting, from the definition of eq:ex1."""
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    k1 = np.asarray(k1, dtype=np.float64)
    k2 = np.asarray(k2, dtype=np.float64)
    val = x1 * k1 + x2 * k2
    if ph.kind == ELLIPSE:
        s1, s2 = np.sin(2 * np.pi * x1), np.sin(2 * np.pi * x2)
        co1, co2 = np.cos(2 * np.pi * x1), np.cos(2 * np.pi * x2)
        c1 = ph.a1 * (2.0 + (1.0 + ph.eta1) * s1 * s2) / 3.0
        c2 = ph.a2 * (2.0 + (1.0 + ph.eta2) * co1 * co2) / 3.0
        val = val + np.sqrt((c1 * k1) ** 2 + (c2 * k2) ** 2)
    return val


def cis_np(phi):
    """exp(2 pi i phi) after an exact FP64 reduction of phi mod 1."""
    r = phi - np.rint(phi)
    return np.exp(2j * np.pi * r)


def grids(N: int):
    """(x1, x2) of X as (N*N,) arrays in row order and (k1, k2) of Omega."""
    i = np.arange(N)
    x1, x2 = np.meshgrid(i / N, i / N, indexing="ij")
    k = np.arange(N) - N // 2
    k1, k2 = np.meshgrid(k, k, indexing="ij")
    return x1.ravel(), x2.ravel(), k1.ravel().astype(np.float64), k2.ravel().astype(np.float64)


def forward_np(N: int, ph: Phase, f: np.ndarray, rows=None) -> np.ndarray:
    x1, x2, k1, k2 = grids(N)
    f = np.asarray(f, dtype=np.complex128).reshape(-1)
    rows = np.arange(N * N) if rows is None else np.asarray(rows)
    out = np.empty(len(rows), dtype=np.complex128)
    for j, r in enumerate(rows):
        out[j] = np.dot(cis_np(phi_np(ph, x1[r], x2[r], k1, k2)), f)
    return out


def adjoint_np(N: int, ph: Phase, u: np.ndarray, cols=None) -> np.ndarray:
    x1, x2, k1, k2 = grids(N)
    u = np.asarray(u, dtype=np.complex128).reshape(-1)
    cols = np.arange(N * N) if cols is None else np.asarray(cols)
    out = np.empty(len(cols), dtype=np.complex128)
    for j, c in enumerate(cols):
        out[j] = np.dot(np.conj(cis_np(phi_np(ph, x1, x2, k1[c], k2[c]))), u)
    return out


def dense_matrix(N: int, ph: Phase) -> np.ndarray:
    """The full N^2 x N^2 kernel K[x, k] = exp(2 pi i Phi(x,k)) (tiny N only)."""
    x1, x2, k1, k2 = grids(N)
    return cis_np(phi_np(ph, x1[:, None], x2[:, None], k1[None, :], k2[None, :]))


def rel_err(u_exact: np.ndarray, u_approx: np.ndarray) -> float:
    """eq:err (Sec. 5): sqrt(sum |u - u^a|^2 / sum |u|^2) over the sample."""
    u_exact = np.asarray(u_exact).reshape(-1)
    u_approx = np.asarray(u_approx).reshape(-1)
    return float(np.sqrt(np.sum(np.abs(u_exact - u_approx) ** 2) / np.sum(np.abs(u_exact) ** 2)))
