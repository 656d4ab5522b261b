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


def test_restricted_sources_equal_the_full_adjoint():
    # the adjoint computed only over the ancestors of some source boxes gives
    # the same values at the sources inside those boxes, zero elsewhere, for
    # every s from 0 to 3 (each level kind present at least once)
    from oracle.butterfly import box_of
    for N, q, s in ((16, 4, 0), (32, 4, 1), (64, 5, 2), (64, 5, 3), (256, 4, 3)):
        m = ButterflyModel(N, q, D.Phase(a1=1.05, a2=0.9), s=s)
        u = white_noise(N, 4)
        full = m.adjoint(u).ravel()
        lB = m.L - m.s
        nb = 1 << lB
        rng = np.random.default_rng(N + s)
        src = [tuple(int(v) for v in rng.integers(0, nb, 2)) for _ in range(3)] + [(0, 0), (nb - 1, nb - 1)]
        part = m.adjoint(u, sources=src).ravel()
        b1, b2 = box_of(m.p1, lB), box_of(m.p2, lB)
        mask = np.zeros(N * N, dtype=bool)
        for c1, c2 in src:
            mask |= (b1 == c1) & (b2 == c2)
        assert mask.any()
        assert np.abs(part[mask] - full[mask]).max() <= 1e-13 * np.abs(full[mask]).max(), (N, q, s)
        assert not np.any(part[~mask])


def _err_s3(q, model=ButterflyModel):
    """eq:err of the step model at the benchmark's schedule depth: N = 256,
    s = 3 (recursion from level L-3 of T_P to level 3, as the numerical
    section runs it), lm = 4 -- initialisation, one p-level, the switch, one
    x-level and the termination over 4^3 boxes B -- with the Fourier phase,
    on two target boxes (128 points) against the direct sum there."""
    N = 256
    f = white_noise(N, 1)
    side = 8
    targets = [(1, 2), (31, 5)]
    rows = np.array([(a1 * side + i) * N + a2 * side + j for a1, a2 in targets
                     for i in range(side) for j in range(side)])
    m = model(N, q, FOURIER)
    assert (m.s, m.lm) == (3, 4)
    u = m.apply(f, targets=targets)
    return D.rel_err(D.forward(N, FOURIER, f, rows), u.ravel()[rows])


def test_spectral_convergence_at_s3():
    # 2^s = 8 termination grid columns and 64 boxes B: a slip that confuses
    # 2^s with 2s or 4^s with 2^s is invisible at s = 1, 2 and O(1) here
    errs = [_err_s3(q) for q in (9, 13, 17, 21)]
    assert all(b < a / 30 for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-8, errs


class _TermGrid2s(ButterflyModel):
    """Termination interpolating at j/(2s) - 1/2 instead of j/2^s - 1/2: the
    same points at s = 1 and s = 2."""
    def term_interp(self):
        from oracle.butterfly import lagrange
        xi = np.arange(1 << self.s) / (2 * self.s) - 0.5
        return lagrange(xi, self.z)


def test_planted_mistake_visible_only_at_s3():
    for s in (1, 2):
        good = _err(32, 9, FOURIER, s=s)
        assert _err(32, 9, FOURIER, s=s, model=_TermGrid2s) == good
    good, bad = _err_s3(13), _err_s3(13, model=_TermGrid2s)
    assert good < 1e-3
    assert bad > 100 * good, (good, bad)
