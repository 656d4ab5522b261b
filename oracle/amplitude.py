"""Variable amplitude a(x,k) for the FIO (TEST INFRASTRUCTURE ONLY: only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import this module; the product path never does).

eq:allfio carries an amplitude a(x,k) in front of the oscillatory kernel.
The end of Sec. 4 reduces it to the unit-amplitude butterfly through a
separated approximation a(x,k) ~ sum_t g_t(x) h_t(k): then

    sum_k a(x,k) e^{2 pi i Phi(x,k)} f(k) = sum_t g_t(x) sum_k e^{2 pi i Phi(x,k)} (h_t f)(k),

i.e. one butterfly application per term, on the input h_t f, scaled by g_t
at the output.  Two references are here:

  * ``dense_forward`` / ``dense_adjoint``: the definition written out, with
    a(x,k) formed as a full matrix from the factors and multiplied into the
    dense kernel (tiny N only);
  * ``separated_forward`` / ``separated_adjoint``: the reduction above on a
    given (FP64 oracle) butterfly model, one term at a time.

Arrays: f, u are (N, N) (x grid in row order / frequency grid k + N/2);
g, h are (rank, N, N) on the same grids as u and f respectively.
"""
import numpy as np

from . import direct as D


def amplitude_matrix(g: np.ndarray, h: np.ndarray) -> np.ndarray:
    """a[x, k] = sum_t g_t(x) h_t(k) as an N^2 x N^2 matrix."""
    rank = g.shape[0]
    return g.reshape(rank, -1).T @ h.reshape(rank, -1)


def dense_forward(N: int, ph: D.Phase, f, g, h) -> np.ndarray:
    """u(x) = sum_k a(x,k) exp(2 pi i Phi(x,k)) f(k) (eq:allfio, dense)."""
    K = D.dense_matrix(N, ph) * amplitude_matrix(g, h)
    return (K @ f.ravel()).reshape(N, N)


def dense_adjoint(N: int, ph: D.Phase, u, g, h) -> np.ndarray:
    """f(k) = sum_x conj(a(x,k) exp(2 pi i Phi(x,k))) u(x) (dense)."""
    K = D.dense_matrix(N, ph) * amplitude_matrix(g, h)
    return (K.conj().T @ u.ravel()).reshape(N, N)


def separated_forward(model, f, g, h) -> np.ndarray:
    """sum_t g_t . B(h_t . f) with B the butterfly ``model`` (end of Sec. 4)."""
    return sum(g[t] * model.apply(h[t] * f) for t in range(g.shape[0]))


def separated_adjoint(model, u, g, h) -> np.ndarray:
    """sum_t conj(h_t) . B^H(conj(g_t) . u), the adjoint of ``separated_forward``."""
    return sum(np.conj(h[t]) * model.adjoint(np.conj(g[t]) * u) for t in range(g.shape[0]))
