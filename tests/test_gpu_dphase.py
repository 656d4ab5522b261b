"""Derivatives of the butterfly with respect to the velocity scalings (a1, a2)
of the ellipse phase (fio_apply_dphase) and the autograd path built on them.

The reference is the FP64 oracle butterfly itself, differentiated by central
finite differences in a1 and a2 (step h = 1e-6 relative): the truncation
error is ~ h^2 (2 pi N)^2 / 6 < 1e-8 relative for N <= 64 and the FP64
rounding noise ~ 1e-16 / h, so the difference quotient is good to ~1e-8,
independent of the GPU path's analytic product-rule formulas.

Tolerances (relative l2 over all outputs): FP64 path 1e-6 (the difference
quotient's own error, with margin); FP32 path: see FP32_TOL -- the derivative
terms 2 pi i rho dG . w are formed from the same FP32 weights as the primal,
so their relative error is that of the primal path.
"""
import functools

import numpy as np
import pytest
import torch

from oracle import direct as D
from oracle.butterfly import ButterflyModel
from workloads import white_noise

from gpu_helpers import rel_l2, rel_max

pytestmark = pytest.mark.gpu

FD_TOL = 1e-6
FP32_TOL = 5e-5

# (N, q, phase, s, lm)
CASES = [
    (16, 5, D.Phase(a1=1.1, a2=0.9), None, None),
    (32, 6, D.Phase(a1=1.1, a2=0.9, eta1=0.2, eta2=0.1), 1, 3),   # even q, other switch level
    (32, 7, D.Phase(), 1, 2),                                      # p-level 2, x-levels 3, 4
    (64, 9, D.Phase(), 2, None),                                   # q of the eq:ex1 workload
    (64, 4, D.Phase(a1=0.9, a2=1.2, eta1=-0.3), 0, None),          # s = 0: Sec. 4 verbatim
    (16, 12, D.Phase(a1=1.3, a2=0.7), None, None),                 # largest q of the tangent path
]


def _ids(c):
    N, q, ph, s, lm = c
    return f"N{N}-q{q}-a{ph.a1}-{ph.a2}-s{s}-lm{lm}"


def _with(ph, **kw):
    d = dict(kind=ph.kind, a1=ph.a1, a2=ph.a2, eta1=ph.eta1, eta2=ph.eta2)
    d.update(kw)
    return D.Phase(**d)


@functools.lru_cache(maxsize=None)
def oracle_fd(N, q, ph, s, lm, seed, h=1e-6):
    """u and the central difference quotients of the FP64 oracle butterfly in a1, a2."""
    f = white_noise(N, seed)
    u = ButterflyModel(N, q, ph, s=s, lm=lm).apply(f)
    out = [u]
    for name in ("a1", "a2"):
        a = getattr(ph, name)
        up = ButterflyModel(N, q, _with(ph, **{name: a * (1 + h)}), s=s, lm=lm).apply(f)
        um = ButterflyModel(N, q, _with(ph, **{name: a * (1 - h)}), s=s, lm=lm).apply(f)
        out.append((up - um) / (2 * a * h))
    return tuple(out)


def _plan(N, q, ph, s, lm, dtype, nrhs_max=1):
    import paper_0809_0719_amd as fio
    return fio.Plan(N, q, fio.Phase(ph.kind, ph.a1, ph.a2, ph.eta1, ph.eta2), s=s, lm=lm, dtype=dtype,
                    nrhs_max=nrhs_max)


def _dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_dphase_matches_oracle_differences_fp64(case):
    N, q, ph, s, lm = case
    u_ref, d1_ref, d2_ref = oracle_fd(N, q, ph, s, lm, 1)
    plan = _plan(N, q, ph, s, lm, torch.complex128)
    u, d1, d2 = (x.cpu().numpy() for x in plan.apply_dphase(_dev(white_noise(N, 1), torch.complex128)))
    errs = [rel_l2(u, u_ref), rel_l2(d1, d1_ref), rel_l2(d2, d2_ref)]
    print(f"dphase fp64 {case}: u {errs[0]:.2e} d/da1 {errs[1]:.2e} d/da2 {errs[2]:.2e}")
    assert errs[0] <= 1e-10
    assert errs[1] <= FD_TOL and errs[2] <= FD_TOL


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_dphase_matches_oracle_differences_fp32(case):
    N, q, ph, s, lm = case
    u_ref, d1_ref, d2_ref = oracle_fd(N, q, ph, s, lm, 1)
    plan = _plan(N, q, ph, s, lm, torch.complex64)
    u, d1, d2 = (x.cpu().numpy() for x in plan.apply_dphase(_dev(white_noise(N, 1), torch.complex64)))
    errs = [rel_l2(u, u_ref), rel_l2(d1, d1_ref), rel_l2(d2, d2_ref)]
    print(f"dphase fp32 {case}: u {errs[0]:.2e} d/da1 {errs[1]:.2e} d/da2 {errs[2]:.2e}")
    assert max(errs) <= FP32_TOL


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-6)])
def test_dphase_primal_equals_apply(dtype, tol):
    N, q, ph = 64, 9, D.Phase(a1=1.05, a2=0.95, eta1=0.1)
    plan = _plan(N, q, ph, None, None, dtype)
    f = _dev(white_noise(N, 7), dtype)
    u_apply = plan.apply(f).cpu().numpy()
    u, _, _ = plan.apply_dphase(f)
    e = rel_max(u.cpu().numpy(), u_apply)
    print(f"primal of the tangent pass vs fio_apply {dtype}: {e:.2e}")
    assert e <= tol


def test_dphase_fourier_is_zero():
    import paper_0809_0719_amd as fio
    N, q = 32, 6
    plan = fio.Plan(N, q, fio.Phase(kind=fio.FOURIER), dtype=torch.complex128)
    f = _dev(white_noise(N, 2), torch.complex128)
    u, d1, d2 = plan.apply_dphase(f)
    assert torch.count_nonzero(d1).item() == 0 and torch.count_nonzero(d2).item() == 0
    assert rel_l2(u.cpu().numpy(), plan.apply(f).cpu().numpy()) <= 1e-12


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_dphase_several_rhs_and_workspace_reuse(dtype):
    """Three right-hand sides at once equal one at a time, with the lazily
    allocated tangent workspace (nrhs_max = 1) and with the plan's own weight
    buffers (nrhs_max = 4); the primal output may be omitted."""
    N, q, ph = 32, 7, D.Phase(a1=1.2, a2=0.8, eta2=0.3)
    f = _dev(white_noise(N, 11, nrhs=3), dtype)
    p1 = _plan(N, q, ph, None, None, dtype, nrhs_max=1)
    p4 = _plan(N, q, ph, None, None, dtype, nrhs_max=4)
    _, a1, a2 = p1.apply_dphase(f, primal=False)
    u4, b1, b2 = p4.apply_dphase(f)
    for r in range(3):
        _, c1, c2 = p1.apply_dphase(f[r])
        assert torch.equal(c1, a1[r]) and torch.equal(c2, a2[r])
    tol = 1e-12 if dtype == torch.complex128 else 1e-6
    assert rel_max(b1.cpu().numpy(), a1.cpu().numpy()) <= tol
    assert rel_max(b2.cpu().numpy(), a2.cpu().numpy()) <= tol
    assert rel_max(u4.cpu().numpy(), p4.apply(f).cpu().numpy()) <= tol


@pytest.mark.parametrize("dtype,N,q,s", [(torch.complex64, 64, 9, 1), (torch.complex128, 64, 9, 1),
                                          (torch.complex64, 32, 12, 1), (torch.complex128, 32, 12, 1),
                                          (torch.complex64, 32, 5, 1), (torch.complex64, 32, 6, 1)])
def test_dphase_batched_levels_equal_one_at_a_time(dtype, N, q, s):
    """A plan with nrhs_max = 9 takes the tangent in chunks of three right-hand
    sides (three weight planes each); seven of them (chunks 3, 3, 1) through
    the batched level and switch kernels give bit for bit what one at a time
    gives, with two p-levels and two x-levels on the path; odd and even q
    (the switch's middle node row, the levels' paired passes)."""
    ph = D.Phase(a1=1.1, a2=0.85, eta1=0.2)
    f = _dev(white_noise(N, 21, nrhs=7), dtype)
    p9 = _plan(N, q, ph, s, None, dtype, nrhs_max=9)
    p1 = _plan(N, q, ph, s, None, dtype, nrhs_max=1)
    u9, b1, b2 = p9.apply_dphase(f)
    for r in range(7):
        u, c1, c2 = p1.apply_dphase(f[r])
        assert torch.equal(u, u9[r]) and torch.equal(c1, b1[r]) and torch.equal(c2, b2[r]), r
    # and the chunked pass is right, not only self-consistent: the last
    # right-hand side (a chunk of one) against the oracle's difference quotients
    fr = white_noise(N, 21, nrhs=7)[6]
    ref = []
    for name in ("a1", "a2"):
        a, h = getattr(ph, name), 1e-6
        up = ButterflyModel(N, q, _with(ph, **{name: a * (1 + h)}), s=s).apply(fr)
        um = ButterflyModel(N, q, _with(ph, **{name: a * (1 - h)}), s=s).apply(fr)
        ref.append((up - um) / (2 * a * h))
    errs = [rel_l2(b1[6].cpu().numpy(), ref[0]), rel_l2(b2[6].cpu().numpy(), ref[1])]
    print(f"batched dphase {dtype} N={N} q={q}: d/da1 {errs[0]:.2e} d/da2 {errs[1]:.2e}")
    assert max(errs) <= (FD_TOL if dtype == torch.complex128 else FP32_TOL)


def test_dphase_bad_arguments():
    import paper_0809_0719_amd as fio
    N = 16
    f = _dev(white_noise(N, 1), torch.complex64)
    plan = fio.Plan(N, 13, fio.Phase())
    with pytest.raises(RuntimeError, match="q <= 12"):
        plan.apply_dphase(f)
    plan = fio.Plan(N, 5, fio.Phase())
    lib = fio.load_library()
    d = torch.empty_like(f)
    assert lib.fio_apply_dphase(plan._h, f.data_ptr(), None, None, d.data_ptr(), 1, None) == -1
    assert lib.fio_apply_dphase(plan._h, f.data_ptr(), None, d.data_ptr(), d.data_ptr(), 1, None) == -1
    assert lib.fio_apply_dphase(plan._h, f.data_ptr(), d.data_ptr(), d.data_ptr(), f.data_ptr(), 1, None) == -1
    assert lib.fio_apply_dphase(plan._h, f.data_ptr(), None, d.data_ptr(), torch.empty_like(f).data_ptr(), 0,
                                None) == -1


def test_phase_gradient_autograd_matches_oracle():
    """d/da of L = ||B(a) f - y||^2 through fio_apply(f, plan, a) against the
    same loss on the FP64 oracle butterfly, differenced in a1 and a2; the
    gradient for f is the adjoint as before."""
    import paper_0809_0719_amd as fio
    N, q = 32, 7
    ph = D.Phase(a1=1.1, a2=0.9, eta1=0.15, eta2=-0.2)
    fn, yn = white_noise(N, 21), white_noise(N, 22)
    plan = _plan(N, q, ph, None, None, torch.complex128)
    a = torch.tensor([ph.a1, ph.a2], dtype=torch.float64, requires_grad=True)
    f = _dev(fn, torch.complex128).requires_grad_(True)
    y = _dev(yn, torch.complex128)
    loss = (fio.fio_apply(f, plan, a) - y).abs().pow(2).sum()
    loss.backward()

    def oracle_loss(a1, a2):
        u = ButterflyModel(N, q, _with(ph, a1=a1, a2=a2)).apply(fn)
        return float(np.sum(np.abs(u - yn) ** 2))

    h = 1e-6
    want = [(oracle_loss(ph.a1 + h, ph.a2) - oracle_loss(ph.a1 - h, ph.a2)) / (2 * h),
            (oracle_loss(ph.a1, ph.a2 + h) - oracle_loss(ph.a1, ph.a2 - h)) / (2 * h)]
    got = a.grad.numpy()
    print(f"grad a: {got} vs oracle differences {want}")
    assert np.allclose(got, want, rtol=1e-6, atol=0)
    assert abs(loss.item() - oracle_loss(ph.a1, ph.a2)) <= 1e-10 * loss.item()
    g_adj = 2 * plan.adjoint(plan.apply(f.detach()) - y)
    assert rel_l2(f.grad.cpu().numpy(), g_adj.cpu().numpy()) <= 1e-12


def test_phase_gradient_descent_recovers_velocity_scaling():
    """Gradient steps on (a1, a2) from a perturbed start, with the step length
    L / ||grad L||^2 (the misfit's minimum is 0), drive the misfit to data
    made with the butterfly at the true scalings down monotonically (FP32).
    On the FP64 oracle butterfly this iteration divides the misfit by ~4 per
    step from the same start."""
    import paper_0809_0719_amd as fio
    N, q = 64, 7
    true = fio.Phase(a1=1.0, a2=1.0)
    plan = fio.Plan(N, q, true)
    f = _dev(white_noise(N, 31), torch.complex64) * 1e-2
    y = plan.apply(f)
    a = torch.tensor([1.0 + 2e-3, 1.0 - 1.5e-3], dtype=torch.float64, requires_grad=True)
    losses = []
    for _ in range(8):
        a.grad = None
        loss = (fio.fio_apply(f, plan, a) - y).abs().pow(2).sum()
        loss.backward()
        losses.append(loss.item())
        with torch.no_grad():
            a -= loss.item() / float(a.grad.pow(2).sum()) * a.grad
    print("misfit:", [f"{v:.3e}" for v in losses], "a:", a.detach().numpy())
    assert all(b < a_ for a_, b in zip(losses, losses[1:]))
    assert losses[-1] < 1e-3 * losses[0]
    assert np.abs(a.detach().numpy() - 1.0).max() < 1e-4


def test_dphase_at_the_benchmark_size():
    """The benchmark's configuration: N = 1024, q = 9, eq:ex1, complex64, a
    plan of nrhs_max = 64 and 64 right-hand sides (chunks of 16 through the
    paired level kernels and the register-table switch).  Properties that hold
    at any size: the primal plane equals fio_apply's batched forward to FP32
    rounding for every right-hand side, and the first and last right-hand
    sides equal the single-right-hand-side pass bit for bit (which the small
    cases above pin to the oracle's difference quotients)."""
    N, q, R = 1024, 9, 64
    ph = D.Phase()
    plan = _plan(N, q, ph, None, None, torch.complex64, nrhs_max=R)
    f = _dev(white_noise(N, 31, nrhs=R), torch.complex64)
    u, d1, d2 = plan.apply_dphase(f)
    ua = plan.apply(f)
    err = max(rel_max(u[r].cpu().numpy(), ua[r].cpu().numpy()) for r in (0, 17, 40, 63))
    print(f"dphase N=1024 q=9 64 RHS: primal vs fio_apply {err:.2e}")
    # two FP32 paths (dense passes here, symmetric passes and matrix cores
    # there), each within 8e-5 relative max of the FP64 model
    assert err <= 1.6e-4
    for r in (0, R - 1):
        u1, c1, c2 = plan.apply_dphase(f[r])
        assert torch.equal(u1, u[r]) and torch.equal(c1, d1[r]) and torch.equal(c2, d2[r]), r
    assert torch.isfinite(d1).all() and torch.isfinite(d2).all()
    assert torch.count_nonzero(d1).item() > 0.99 * d1.numel()
