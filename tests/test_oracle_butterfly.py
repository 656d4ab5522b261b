"""Pins of the FP64 step model of the butterfly (Sec. 4) against facts that
do not come from the model itself:

* spectral convergence to the direct sum (eq:dfio) as q grows, for the
  Fourier phase and for eq:ex1 -- a wrong sign, index, transposition or
  dropped factor anywhere in the five steps leaves an O(1) error;
* the adjoint is the exact conjugate transpose (dot-product identity and a
  dense check), and the map is linear;
* planted mistakes in the model are caught by these pins.
"""
import numpy as np
import pytest

from oracle import direct as D
from oracle.butterfly import ButterflyModel
from workloads import white_noise

FOURIER = D.Phase(kind=D.FOURIER)
ELLIPSE = D.Phase()


def _err(N, q, ph, s=None, lm=None, seed=1, model=ButterflyModel):
    f = white_noise(N, seed)
    ub = model(N, q, ph, s=s, lm=lm).apply(f)
    return D.rel_err(D.forward(N, ph, f), ub)


def test_fourier_spectral_convergence_all_steps():
    # N=32, s=1: init, p-level 2, switch at 2, x-levels 3 and 4, termination
    errs = [_err(32, q, FOURIER, s=1) for q in (9, 13, 17, 21)]
    assert all(b < a / 10 for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-7, errs


def test_ellipse_spectral_convergence():
    # eq:ex1 (constant amplitude) at N=8: the residual phase of a box pair is
    # large for this phase, so convergence sets in at higher q
    errs = [_err(8, q, ELLIPSE) for q in (17, 33, 41)]
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[-1] < 2e-5, errs


def test_ellipse_with_levels_converges():
    e = _err(16, 33, D.Phase(a1=1.05, a2=0.95, eta1=0.1, eta2=0.2), s=1)
    assert e < 2e-3


def test_odd_levels_and_switch_choices_agree():
    # L odd: both readings of the switch level converge to the same operator
    for lm in (2, 3):
        assert _err(32, 19, FOURIER, s=1, lm=lm) < 5e-5


def test_adjoint_identity_and_linearity():
    for N, q, s in ((32, 7, 1), (32, 5, 2), (64, 5, 3)):
        m = ButterflyModel(N, q, ELLIPSE, s=s)
        f, u = white_noise(N, 3), white_noise(N, 4)
        Bf = m.apply(f)
        BHu = m.adjoint(u)
        lhs, rhs = np.vdot(u, Bf), np.vdot(BHu, f)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
        g = white_noise(N, 5)
        a, b = 0.7 - 0.2j, -1.3 + 0.4j
        assert np.abs(m.apply(a * f + b * g) - (a * Bf + b * m.apply(g))).max() <= 1e-12 * np.abs(Bf).max()


def test_adjoint_dense_conjugate_transpose():
    N, q = 8, 5
    m = ButterflyModel(N, q, ELLIPSE)
    E = np.eye(N * N).reshape(N * N, N, N)
    B = np.stack([m.apply(e).ravel() for e in E], axis=1)          # columns B e_j
    BH = np.stack([m.adjoint(e).ravel() for e in E], axis=1)
    assert np.abs(BH - B.conj().T).max() <= 1e-13 * np.abs(B).max()


# ---- planted mistakes: each must be caught by the convergence pin ---------

class _ConjSwitch(ButterflyModel):
    def switch_kernel(self, a1, a2):
        return np.conj(super().switch_kernel(a1, a2))


class _TransposedX(ButterflyModel):
    def x_interp(self, l):
        return np.swapaxes(super().x_interp(l), 1, 2)


class _TransposedP(ButterflyModel):
    def p_interp(self, lB):
        return np.swapaxes(super().p_interp(lB), 2, 3)


class _ShiftedTerm(ButterflyModel):
    def term_interp(self):
        xi = (np.arange(1 << self.s) + 0.5) / (1 << self.s) - 0.5   # wrong grid points
        from oracle.butterfly import lagrange
        return lagrange(xi, self.z)


class _WrongPolar(ButterflyModel):
    def E_p(self, x1, x2, p1, p2):
        return super().E_p(x1, x2, p1, np.asarray(p2) + 1.0 / self.N)


@pytest.mark.parametrize("mutant", [_ConjSwitch, _TransposedX, _TransposedP, _ShiftedTerm, _WrongPolar])
def test_planted_mistakes_are_caught(mutant):
    good = _err(32, 13, FOURIER, s=1)
    bad = _err(32, 13, FOURIER, s=1, model=mutant)
    assert good < 1e-3
    assert bad > 100 * good, (good, bad)


def test_restricted_targets_equal_the_full_pass():
    # computing only the ancestor chain of some target boxes gives the same
    # potentials on those boxes and the same weights for those ancestors
    N, q, s = 64, 5, 2
    m = ButterflyModel(N, q, ELLIPSE, s=s)
    f = white_noise(N, 9)
    u_full, lev_full = m.apply(f, return_levels=True)
    targets = [(0, 0), (5, 11), (15, 15)]
    u_part, lev_part = m.apply(f, return_levels=True, targets=targets)
    m_side = 1 << s
    for a1, a2 in targets:
        blk = (slice(a1 * m_side, (a1 + 1) * m_side), slice(a2 * m_side, (a2 + 1) * m_side))
        assert np.array_equal(u_part[blk], u_full[blk])
    for key, part in lev_part.items():
        for (a1, a2), w in part.items():
            assert np.array_equal(w, lev_full[key][a1, a2])
