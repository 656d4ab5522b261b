"""The autograd wrapper: backward of u = B f is the adjoint butterfly.

PyTorch's convention for a real loss L of complex f returns
grad_f = dL/d(conj f) * 2, so for L = ||B f - y||^2 the gradient is
2 B^H (B f - y) and dL = Re <grad_f, df> for a perturbation df."""
import numpy as np
import pytest
import torch

from oracle import direct as D
from oracle.butterfly import ButterflyModel
from workloads import velocity_scalings, white_noise

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


def _plan(N, q, dtype):
    import paper_0809_0719_amd as fio
    return fio.Plan(N, q, fio.Phase(a1=1.05, a2=0.95), dtype=dtype)


def test_gradient_is_the_adjoint_and_matches_dense_fp64():
    import paper_0809_0719_amd as fio
    N, q = 8, 5
    plan = _plan(N, q, torch.complex128)
    f = _dev(white_noise(N, 1), torch.complex128).requires_grad_(True)
    y = _dev(white_noise(N, 2), torch.complex128)
    loss = (fio.fio_apply(f, plan) - y).abs().pow(2).sum()
    loss.backward()
    # dense FP64 butterfly matrix from the oracle model (columns B e_j)
    m = ButterflyModel(N, q, D.Phase(a1=1.05, a2=0.95))
    E = np.eye(N * N).reshape(N * N, N, N)
    B = np.stack([m.apply(e).ravel() for e in E], axis=1)
    fn = white_noise(N, 1).ravel()
    want = 2 * B.conj().T @ (B @ fn - white_noise(N, 2).ravel())
    got = f.grad.cpu().numpy().ravel()
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


@pytest.mark.parametrize("dtype,h,tol", [(torch.complex128, 1e-6, 1e-7), (torch.complex64, 1e-2, 2e-3)])
def test_gradient_matches_finite_differences(dtype, h, tol):
    import paper_0809_0719_amd as fio
    N, q = 64, 7
    plan = _plan(N, q, dtype)
    f0 = _dev(white_noise(N, 3), dtype)
    y = _dev(white_noise(N, 4), dtype) * 10
    v = _dev(white_noise(N, 5), dtype)

    def L(f):
        return (fio.fio_apply(f, plan) - y).abs().pow(2).sum()

    f = f0.clone().requires_grad_(True)
    L(f).backward()
    dir_grad = torch.real(torch.vdot(f.grad.flatten(), v.flatten())).item()
    with torch.no_grad():
        fd = (L(f0 + h * v).item() - L(f0 - h * v).item()) / (2 * h)
    assert abs(fd - dir_grad) <= tol * abs(dir_grad), (fd, dir_grad)


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-10), (torch.complex64, 2e-5)])
def test_gradients_against_dense_fp64_columns_n64(dtype, tol):
    """The differentiable apply at its check size: N = 64, q = 9, s = 2 (so the
    schedule has a p-level, the switch and an x-level), velocity scalings
    a ~ U[0.8, 1.2]^2 (seed 5), loss ||B(a) f - u*||^2 with u* = B(a) f* from
    the FP64 oracle (f seed 3, f* seed 4).

    grad_f: the whole vector against 2 B^H (B f - u*) from the oracle's
    forward and adjoint, and 24 sampled entries against dense columns of the
    FP64 butterfly matrix: entry j is 2 <B e_j, B f - u*>, B e_j an oracle
    forward of the unit vector e_j (no adjoint involved).
    grad_a: against 2 Re <B f - u*, dB/da_k f>, the derivative a central
    difference of the oracle butterfly in a_k (relative step 1e-6)."""
    import paper_0809_0719_amd as fio
    N, q, s, h = 64, 9, 2, 1e-6
    a1, a2 = velocity_scalings(5)
    ph = D.Phase(a1=a1, a2=a2)
    m = ButterflyModel(N, q, ph, s=s)
    f, fstar = white_noise(N, 3), white_noise(N, 4)
    if dtype == torch.complex64:  # the oracle sees the values the library stores
        f = f.astype(np.complex64).astype(np.complex128)
    ustar = m.apply(fstar)
    res = m.apply(f) - ustar
    plan = fio.Plan(N, q, fio.Phase(a1=a1, a2=a2), s=s, dtype=dtype)
    fd = _dev(f, dtype).requires_grad_(True)
    a = torch.tensor([a1, a2], dtype=torch.float64, requires_grad=True)
    loss = (fio.fio_apply(fd, plan, a) - _dev(ustar, dtype)).abs().pow(2).sum()
    loss.backward()
    got = fd.grad.cpu().numpy().astype(np.complex128)
    want = 2 * m.adjoint(res)
    e_vec = np.linalg.norm(got - want) / np.linalg.norm(want)
    rng = np.random.default_rng(17)
    cols = rng.choice(N * N, size=24, replace=False)
    worst = 0.0
    scale = np.abs(want).max()
    for j in cols:
        e = np.zeros(N * N, dtype=np.complex128)
        e[j] = 1.0
        col = m.apply(e.reshape(N, N)).ravel()
        wj = 2 * np.vdot(col, res.ravel())
        worst = max(worst, abs(got.ravel()[j] - wj) / scale)
    ga = []
    for name, av in (("a1", a1), ("a2", a2)):
        kw = dict(a1=a1, a2=a2)
        kw[name] = av * (1 + h)
        up = ButterflyModel(N, q, D.Phase(**kw), s=s).apply(f)
        kw[name] = av * (1 - h)
        um = ButterflyModel(N, q, D.Phase(**kw), s=s).apply(f)
        ga.append(2 * np.real(np.vdot(res, (up - um) / (2 * av * h))))
    e_a = np.abs(a.grad.numpy() - np.array(ga)).max() / np.abs(ga).max()
    print(f"N={N} q={q} s={s} {dtype}: grad_f vs oracle adjoint {e_vec:.2e}, "
          f"vs dense columns {worst:.2e}; grad_a {a.grad.numpy()} vs {np.array(ga)} ({e_a:.2e})")
    assert e_vec <= tol and worst <= tol
    assert e_a <= (1e-6 if dtype == torch.complex128 else 5e-4)
