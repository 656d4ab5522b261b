"""Pins of the direct-sum oracle (eq:dfio) against facts fixed by the
mathematics: the DFT closed form, exact phase values, homogeneity, a lone
source at k = 0, linearity, the dense conjugate transpose, and the agreement
of two independent implementations (C loop and numpy)."""
import math

import numpy as np
import pytest

from oracle import direct as D
from workloads import sample_points, white_noise


def test_fourier_phase_is_the_dft():
    # Phi = x.k with x = i/N: u = N^2 * IDFT(ifftshift(f)) exactly (closed form)
    for N in (8, 16, 32):
        f = white_noise(N, seed=11)
        u = D.forward(N, D.Phase(kind=D.FOURIER), f).reshape(N, N)
        ref = N * N * np.fft.ifft2(np.fft.ifftshift(f))
        assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()


def test_ellipse_phase_hand_values():
    # eq:ex1 at x = (1/4, 1/4): c1 = (2 + 1)/3 = 1, c2 = (2 + 0)/3 = 2/3
    ph = D.Phase()
    want = 7.0 / 4.0 + math.sqrt(145.0) / 3.0          # k = (3, 4)
    assert abs(D.phi_c(ph, 0.25, 0.25, 3.0, 4.0) - want) < 1e-13
    assert abs(float(D.phi_np(ph, 0.25, 0.25, 3.0, 4.0)) - want) < 1e-13
    # x = (0, 0): c1 = 2/3, c2 = (2 + 1)/3 = 1; k = (-5, 2): Phi = sqrt(100/9 + 4)
    want = math.sqrt(100.0 / 9.0 + 4.0)
    assert abs(D.phi_c(ph, 0.0, 0.0, -5.0, 2.0) - want) < 1e-13
    # learnable scalings and modulation amplitudes enter as c_j -> a_j (2 + (1+eta_j) m_j)/3
    ph2 = D.Phase(a1=1.1, a2=0.9, eta1=0.2, eta2=0.1)
    c1 = 1.1 * (2 + 1.2 * 1.0) / 3
    c2 = 0.9 * (2 + 1.1 * 0.0) / 3
    want = 7.0 / 4.0 + math.sqrt((3 * c1) ** 2 + (4 * c2) ** 2)
    assert abs(D.phi_c(ph2, 0.25, 0.25, 3.0, 4.0) - want) < 1e-12


def test_phase_homogeneous_degree_one():
    rng = np.random.default_rng(3)
    ph = D.Phase(a1=1.07, a2=0.93, eta1=0.2, eta2=0.15)
    for _ in range(50):
        x1, x2 = rng.uniform(0, 1, 2)
        k1, k2 = rng.uniform(-50, 50, 2)
        lam = rng.uniform(0.1, 5.0)
        a = D.phi_c(ph, x1, x2, lam * k1, lam * k2)
        b = lam * D.phi_c(ph, x1, x2, k1, k2)
        assert abs(a - b) <= 1e-12 * max(1.0, abs(b))
    assert D.phi_c(ph, 0.3, 0.7, 0.0, 0.0) == 0.0


def test_source_at_zero_frequency_gives_constant():
    N = 16
    f = np.zeros((N, N), complex)
    f[N // 2, N // 2] = 2.5 - 1.0j                     # k = (0, 0)
    u = D.forward(N, D.Phase(), f)
    assert np.abs(u - (2.5 - 1.0j)).max() < 1e-14


def test_single_source_gives_its_kernel():
    N = 16
    f = np.zeros((N, N), complex)
    k1, k2 = 3, -5
    f[k1 + N // 2, k2 + N // 2] = 1.0
    ph = D.Phase()
    u = D.forward(N, ph, f)
    x1, x2, _, _ = D.grids(N)
    want = np.array([np.exp(2j * np.pi * D.phi_c(ph, a, b, k1, k2)) for a, b in zip(x1, x2)])
    assert np.abs(u - want).max() < 1e-12


def test_linearity():
    N = 16
    ph = D.Phase()
    f, g = white_noise(N, 1), white_noise(N, 2)
    a, b = 0.3 - 1.2j, 2.0 + 0.5j
    lhs = D.forward(N, ph, a * f + b * g)
    rhs = a * D.forward(N, ph, f) + b * D.forward(N, ph, g)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_adjoint_is_dense_conjugate_transpose():
    N = 8
    ph = D.Phase(a1=1.1, a2=0.85)
    K = D.dense_matrix(N, ph)                           # built by the numpy twin
    u = white_noise(N, 5)
    f_c = D.adjoint(N, ph, u)
    assert np.abs(f_c - K.conj().T @ u.ravel()).max() <= 1e-12 * np.abs(f_c).max()
    f = white_noise(N, 6)
    lhs = np.vdot(u.ravel(), D.forward(N, ph, f))
    rhs = np.vdot(D.adjoint(N, ph, u), f.ravel())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_c_and_numpy_twins_agree():
    N = 32
    for ph in (D.Phase(), D.Phase(kind=D.FOURIER), D.Phase(a1=0.8, a2=1.2, eta1=0.3, eta2=0.05)):
        f = white_noise(N, 7)
        rows = sample_points(N, 40, seed=8)
        a = D.forward(N, ph, f, rows)
        b = D.forward_np(N, ph, f, rows)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
        c = D.adjoint(N, ph, white_noise(N, 9), rows)
        d = D.adjoint_np(N, ph, white_noise(N, 9), rows)
        assert np.abs(c - d).max() <= 1e-12 * np.abs(c).max()


def test_rel_err_metric():
    # eq:err: sqrt(sum |u - ua|^2 / sum |u|^2)
    u = np.array([3.0 + 4.0j, 0.0])
    ua = np.array([3.0 + 4.0j, 1.0])
    assert D.rel_err(u, ua) == pytest.approx(1.0 / 5.0)
