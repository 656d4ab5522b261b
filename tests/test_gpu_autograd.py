"""The autograd wrapper: backward of u = B f is the adjoint butterfly.

PyTorch's convention for a real loss L of complex f returns
grad_f = dL/d(conj f) * 2, so for L = ||B f - y||^2 the gradient is
2 B^H (B f - y) and dL = Re <grad_f, df> for a perturbation df."""
import numpy as np
import pytest
import torch

from oracle import direct as D
from oracle.butterfly import ButterflyModel
from workloads import white_noise

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
