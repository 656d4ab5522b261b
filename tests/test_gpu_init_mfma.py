"""The initialisation and its adjoint on the matrix cores (complex64 plans
with s = 3 and q <= 9 take this path): stage-0 weights and whole passes
against the FP64 oracle, and several right-hand sides at once against one at
a time (the forward kernel takes them in pairs, so an odd count leaves a
half-filled last pair).  Tolerance as for the other FP32 parity tests: the
contraction sums at most ~200 FP32 products per output, accumulated in FP32
by the MFMA tiles."""
import functools

import numpy as np
import pytest
import torch

from oracle import direct as D
from oracle.butterfly import ButterflyModel
from workloads import white_noise

from gpu_helpers import rel_l2, rel_max, weights_to_oracle

pytestmark = pytest.mark.gpu

FP32_TOL = 2e-5


@functools.lru_cache(maxsize=None)
def _oracle(N, q, ph, seed):
    m = ButterflyModel(N, q, ph)
    u, lev = m.apply(white_noise(N, seed), return_levels=True)
    return m, u, lev


def _plan(N, q, ph, nrhs_max=1):
    import paper_0809_0719_amd as fio
    return fio.Plan(N, q, fio.Phase(ph.kind, ph.a1, ph.a2, ph.eta1, ph.eta2), dtype=torch.complex64,
                    nrhs_max=nrhs_max)


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).to(torch.complex64).cuda()


@pytest.mark.parametrize("q", [3, 4, 5, 6, 8, 9])
def test_mfma_initialisation_matches_oracle(q):
    N, ph = 64, D.Phase(a1=1.1, a2=0.95, eta1=0.1)
    m, _, lev = _oracle(N, q, ph, 1)
    plan = _plan(N, q, ph)
    assert plan.s == 3
    w = weights_to_oracle(plan.debug_stage(_dev(white_noise(N, 1)), 0).cpu().numpy(), N, q, 3)
    e2, em = rel_l2(w, lev["init"]), rel_max(w, lev["init"])
    print(f"init q={q}: rel_l2 {e2:.2e} rel_max {em:.2e}")
    assert e2 <= FP32_TOL and em <= 4 * FP32_TOL


@pytest.mark.parametrize("N,q", [(64, 9), (128, 5), (64, 3)])
def test_mfma_initialisation_whole_pass_both_directions(N, q):
    ph = D.Phase(a1=0.9, a2=1.05, eta2=0.2)
    _, u_ref, _ = _oracle(N, q, ph, 4)
    f_ref = ButterflyModel(N, q, ph).adjoint(white_noise(N, 5))
    plan = _plan(N, q, ph)
    u = plan.apply(_dev(white_noise(N, 4))).cpu().numpy()
    f = plan.adjoint(_dev(white_noise(N, 5))).cpu().numpy()
    eu, ef = rel_l2(u, u_ref), rel_l2(f, f_ref)
    print(f"N={N} q={q}: forward {eu:.2e} adjoint {ef:.2e}")
    assert eu <= FP32_TOL and ef <= FP32_TOL


@pytest.mark.parametrize("nrhs", [2, 3, 5, 17])
def test_mfma_initialisation_batched_equals_one_by_one(nrhs):
    """A box's right-hand sides are split over up to eight workgroups: 17 gives
    the forward nine passes of two (chunks of two passes, the last chunks
    empty) and the adjoint chunks of three right-hand sides (the last two
    empty)."""
    N, q, ph = 64, 9, D.Phase()
    plan = _plan(N, q, ph, nrhs_max=nrhs)
    single = _plan(N, q, ph)
    f = _dev(white_noise(N, 9, nrhs=nrhs))
    u = plan.apply(f)
    g = plan.adjoint(u)
    for r in range(nrhs):
        u1 = single.apply(f[r])
        g1 = single.adjoint(u1)
        assert rel_max(u[r].cpu().numpy(), u1.cpu().numpy()) <= 1e-6
        assert rel_max(g[r].cpu().numpy(), g1.cpu().numpy()) <= 1e-6


def test_mfma_initialisation_empty_and_sparse_boxes():
    """Sources only in a few boxes of T_P (the others empty): the boxes without
    sources must produce exact zeros, and the rest still match the oracle."""
    N, q, ph = 64, 7, D.Phase()
    f = np.zeros((N, N), dtype=np.complex128)
    rng = np.random.default_rng(3)
    k = rng.integers(0, N, size=(40, 2))
    f[k[:, 0], k[:, 1]] = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    m = ButterflyModel(N, q, ph)
    _, lev = m.apply(f, return_levels=True)
    plan = _plan(N, q, ph)
    w = weights_to_oracle(plan.debug_stage(_dev(f), 0).cpu().numpy(), N, q, 3)
    ref = lev["init"]
    empty = np.all(ref == 0, axis=(0, 1, 4, 5))
    assert empty.any()
    assert np.all(w[:, :, empty] == 0)
    assert rel_l2(w, ref) <= FP32_TOL
