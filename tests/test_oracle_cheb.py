"""Pins of the Chebyshev grid and Lagrange basis of Sec. 3 and of the
translation/level invariance of the interpolation matrices (Sec. 4)."""
import numpy as np

from oracle.butterfly import ButterflyModel, cheb_nodes, lagrange
from oracle.direct import Phase


def test_nodes_are_chebyshev_extrema():
    for q in (3, 5, 9, 16):
        z = cheb_nodes(q)
        assert abs(z[0] - 0.5) < 1e-16 and abs(z[-1] + 0.5) < 1e-16
        # extrema of T_{q-1} on [-1/2, 1/2]: |T_{q-1}(2 z_i)| = 1
        assert np.allclose(np.abs(np.cos((q - 1) * np.arccos(2 * z))), 1.0, atol=1e-12)


def test_lagrange_cardinal_partition_and_polynomial_reproduction():
    rng = np.random.default_rng(0)
    for q in (3, 5, 7, 9, 12):
        z = cheb_nodes(q)
        assert np.allclose(lagrange(z, z), np.eye(q), atol=1e-13)
        xi = rng.uniform(-0.5, 0.5, 100)
        Lv = lagrange(xi, z)                                 # (100, q)
        assert np.allclose(Lv.sum(axis=1), 1.0, atol=1e-12)
        for m in range(q):                                   # degree < q is reproduced exactly
            assert np.allclose(Lv @ z ** m, xi ** m, atol=1e-12)
        # degree q is not (the interpolant is of degree q-1)
        assert np.abs(Lv @ z ** q - xi ** q).max() > 1e-10


def test_interpolation_matrices_are_translation_and_level_invariant():
    # L^B_t(p^{B_c}_t') is the same for every box B and level (Sec. 4)
    q = 7
    z = cheb_nodes(q)
    ref = [lagrange((z + c - 0.5) / 2.0, z) for c in (0, 1)]      # (t', t) at child c
    m = ButterflyModel(64, q, Phase())
    for lB in (1, 2, 3, 4, 5):
        nB = 1 << lB
        rng = np.random.default_rng(lB)
        for b in rng.integers(0, nB, 4):
            for c in (0, 1):
                child = 2 * b + c
                cn = (child + 0.5) / (2 * nB) + z / (2 * nB)       # child's nodes, absolute
                loc = (cn - (b + 0.5) / nB) * nB                   # parent-local
                assert np.allclose(lagrange(loc, z), ref[c], atol=1e-12)
    # the same matrices appear in the model's x-interpolation tables
    Xm = m.x_interp(4)
    for a in range(16):
        assert np.allclose(Xm[a], ref[a & 1], atol=1e-12)
