"""Pins of the variable-amplitude oracle (eq:allfio with a separated
amplitude, end of Sec. 4) against facts fixed by the mathematics: a
pure-Python double loop on a tiny grid, the DFT closed form for the Fourier
phase (which fixes the x and k grids of g and h), the unit amplitude, the
dense conjugate transpose, and the agreement of the per-term butterfly
reduction with the dense sum within the butterfly's own error."""
import cmath
import math

import numpy as np
import pytest

from oracle import amplitude as A
from oracle import direct as D
from oracle.butterfly import ButterflyModel
from workloads import white_noise


def _factors(N, rank, seed):
    """Smooth, non-symmetric complex factors on the grids of u (g) and f (h)."""
    rng = np.random.default_rng(seed)
    i = np.arange(N)
    x1, x2 = np.meshgrid(i / N, i / N, indexing="ij")
    k1, k2 = np.meshgrid(i - N // 2, i - N // 2, indexing="ij")
    g = np.empty((rank, N, N), complex)
    h = np.empty((rank, N, N), complex)
    for t in range(rank):
        c = rng.standard_normal(6)
        g[t] = (1 + c[0] * x1 + c[1] * x2 ** 2) * np.exp(1j * (c[2] * x1 - x2))
        h[t] = 1 / (1 + 0.1 * (c[3] * k1 / N) ** 2 + (k2 / N + c[4]) ** 2) * np.exp(1j * c[5] * k1 / N)
    return g, h


def test_dense_matches_python_double_loop():
    N, rank = 4, 2
    ph = D.Phase(a1=1.1, a2=0.9, eta1=0.2)
    f = white_noise(N, 5)
    g, h = _factors(N, rank, 1)
    u = A.dense_forward(N, ph, f, g, h)
    for i1 in range(N):
        for i2 in range(N):
            acc = 0j
            for j1 in range(N):
                for j2 in range(N):
                    a = sum(g[t, i1, i2] * h[t, j1, j2] for t in range(rank))
                    phi = D.phi_c(ph, i1 / N, i2 / N, float(j1 - N // 2), float(j2 - N // 2))
                    acc += a * cmath.exp(2j * math.pi * phi) * f[j1, j2]
            assert abs(u[i1, i2] - acc) <= 1e-12 * max(1.0, abs(acc))


def test_fourier_phase_rank_one_is_scaled_dft():
    # Phi = x.k, a = g(x) h(k): u = g . N^2 IDFT(ifftshift(h f)) exactly
    N = 16
    f = white_noise(N, 7)
    g, h = _factors(N, 1, 2)
    u = A.dense_forward(N, D.Phase(kind=D.FOURIER), f, g, h)
    ref = g[0] * N * N * np.fft.ifft2(np.fft.ifftshift(h[0] * f))
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()
    # adjoint: f = conj(h) . fftshift(DFT(conj(g) v)) exactly
    v = white_noise(N, 8)
    fa = A.dense_adjoint(N, D.Phase(kind=D.FOURIER), v, g, h)
    ref_a = np.conj(h[0]) * np.fft.fftshift(np.fft.fft2(np.conj(g[0]) * v))
    assert np.abs(fa - ref_a).max() <= 1e-12 * np.abs(ref_a).max()


def test_unit_amplitude_is_the_plain_fio():
    N = 8
    ph = D.Phase()
    f = white_noise(N, 9)
    one = np.ones((1, N, N), complex)
    u = A.dense_forward(N, ph, f, one, one)
    ref = D.forward(N, ph, f).reshape(N, N)
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()


def test_dense_adjoint_is_the_conjugate_transpose():
    N, rank = 8, 3
    ph = D.Phase(a1=0.9, a2=1.2, eta2=0.3)
    g, h = _factors(N, rank, 3)
    f, v = white_noise(N, 10), white_noise(N, 11)
    lhs = np.vdot(v, A.dense_forward(N, ph, f, g, h))
    rhs = np.vdot(A.dense_adjoint(N, ph, v, g, h), f)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


class _Exact:
    """The exact unit-amplitude FIO (dense), in the role of the butterfly."""

    def __init__(self, N, ph):
        self.K = D.dense_matrix(N, ph)
        self.N = N

    def apply(self, f):
        return (self.K @ f.ravel()).reshape(self.N, self.N)

    def adjoint(self, u):
        return (self.K.conj().T @ u.ravel()).reshape(self.N, self.N)


def test_separated_reduction_is_exact_with_the_exact_operator():
    """With B the exact FIO the per-term reduction equals the dense sum up to
    rounding (the identity of the end of Sec. 4), for the ellipse phase."""
    N, rank = 8, 4
    ph = D.Phase(a1=1.1, a2=0.9, eta1=0.2, eta2=-0.1)
    g, h = _factors(N, rank, 5)
    f, v = white_noise(N, 14), white_noise(N, 15)
    ex = _Exact(N, ph)
    u = A.separated_forward(ex, f, g, h)
    ref = A.dense_forward(N, ph, f, g, h)
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()
    fa = A.separated_adjoint(ex, v, g, h)
    ref_a = A.dense_adjoint(N, ph, v, g, h)
    assert np.abs(fa - ref_a).max() <= 1e-12 * np.abs(ref_a).max()
    # a plausible mistake (factors on the wrong grids) is caught
    assert np.abs(A.separated_forward(ex, f, h, g) - ref).max() > 0.1 * np.abs(ref).max()


@pytest.mark.parametrize("N,q,tol", [(16, 12, 2e-2), (32, 12, 4e-3)])
def test_separated_butterfly_approaches_dense_sum(N, q, tol):
    """sum_t g_t B(h_t f) with the oracle butterfly against eq:allfio's dense
    sum for the Fourier phase, where the butterfly is accurate (unit-amplitude
    error 5e-3 and 8e-4 at these (N, q)): the difference is the butterfly's
    own error, so swapped or conjugated factors fail by O(1)."""
    rank = 3
    ph = D.Phase(kind=D.FOURIER)
    f, v = white_noise(N, 12), white_noise(N, 13)
    g, h = _factors(N, rank, 4)
    model = ButterflyModel(N, q, ph)
    u = A.separated_forward(model, f, g, h)
    assert D.rel_err(A.dense_forward(N, ph, f, g, h).ravel(), u.ravel()) <= tol
    fa = A.separated_adjoint(model, v, g, h)
    assert D.rel_err(A.dense_adjoint(N, ph, v, g, h).ravel(), fa.ravel()) <= tol
    # the reduction's adjoint is its exact conjugate transpose
    lhs, rhs = np.vdot(v, u), np.vdot(fa, f)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    bad = A.separated_adjoint(model, v, np.conj(g), h)
    assert D.rel_err(A.dense_adjoint(N, ph, v, g, h).ravel(), bad.ravel()) > 0.1
