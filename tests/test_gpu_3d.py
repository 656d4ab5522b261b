"""Three-dimensional butterfly (fio3_*, eq:ex3) against the FP64 3-D oracle
model, for every step of the schedule: N = 8 with s = 0 (a p-level, the
switch, two x-levels), N = 8 with s = 1, N = 16 with s = 1 (p-level 2,
x-level 3) and with the default s = 2 (initialisation, switch and
termination only), N = 4, both phases, q from 3 to 8.

Tolerances: FP64 1e-10 relative (rounding of sums of up to 8 q^3 terms);
FP32 5e-5 relative l2 -- the phases are FP64 and reduced exactly, the
exponentials and the sums FP32, with up to 8 q^3 = 4096 terms per output
(the 2-D bound, 2e-5, scaled by the longer sums)."""
import functools

import numpy as np
import pytest
import torch

from oracle import butterfly3 as B

from gpu_helpers import rel_l2, rel_max

pytestmark = pytest.mark.gpu


def _noise(N, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))) / np.sqrt(2)


@functools.lru_cache(maxsize=None)
def _oracle(N, q, kind, s, lm, seed):
    return B.ButterflyModel3(N, q, kind, s=s, lm=lm).apply(_noise(N, seed))


# (N, q, kind, s, lm)
CASES = [
    (8, 5, B.SPHERES, 0, 1),
    (8, 7, B.FOURIER, 0, 1),
    (8, 3, B.SPHERES, 1, 1),
    (8, 8, B.SPHERES, 1, 2),
    (16, 5, B.SPHERES, 1, 2),
    (16, 4, B.FOURIER, None, None),
    (4, 6, B.SPHERES, None, None),
]


def _ids(c):
    N, q, kind, s, lm = c
    return f"N{N}-q{q}-kind{kind}-s{s}-lm{lm}"


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-10), (torch.complex64, 5e-5)])
@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_3d_matches_oracle(case, dtype, tol):
    import paper_0809_0719_amd as fio
    N, q, kind, s, lm = case
    f = _noise(N, 4)
    plan = fio.Plan3(N, q, kind, s=s, lm=lm, dtype=dtype)
    u = plan.apply(torch.as_tensor(f).to(dtype).cuda()).cpu().numpy()
    u_ref = _oracle(N, q, kind, s, lm, 4)
    e2, em = rel_l2(u, u_ref), rel_max(u, u_ref)
    print(f"3-D {case} {dtype}: l2 {e2:.2e} max {em:.2e}")
    assert e2 <= tol and em <= 4 * tol


def test_3d_approaches_direct_sum_on_the_gpu():
    """N = 32, eq:ex3, q = 7: the butterfly against the oracle's direct sum
    on 128 sampled targets (the estimate eq:err of Sec. 5); the 3-D model's
    error at N = 8, 16 and q = 7 is 0.12-0.14, so a wrong index in any step
    would show as O(1)."""
    import paper_0809_0719_amd as fio
    N, q = 32, 7
    f = _noise(N, 5)
    plan = fio.Plan3(N, q, B.SPHERES, dtype=torch.complex128)
    u = plan.apply(torch.as_tensor(f).cuda()).cpu().numpy().ravel()
    rows = np.random.default_rng(6).choice(N ** 3, size=128, replace=False)
    ref = B.direct3(N, B.SPHERES, f, rows)
    e = float(np.linalg.norm(u[rows] - ref) / np.linalg.norm(ref))
    print(f"3-D N=32 q=7 eq:err on 128 points: {e:.3e}")
    assert e < 0.25


def test_3d_bad_arguments():
    import ctypes
    import paper_0809_0719_amd as fio
    lib = fio.load_library()
    h = ctypes.c_void_p()
    assert lib.fio3_plan(12, 5, 1, -1, -1, fio.C64, ctypes.byref(h)) == -1   # not a power of two
    assert lib.fio3_plan(16, 9, 1, -1, -1, fio.C64, ctypes.byref(h)) == -1   # q > 8
    assert lib.fio3_plan(16, 5, 7, -1, -1, fio.C64, ctypes.byref(h)) == -1   # phase kind
    assert lib.fio3_plan(16, 5, 1, 3, 1, fio.C64, ctypes.byref(h)) == -1     # s > lm
    plan = fio.Plan3(8, 3)
    f = torch.zeros((8, 8, 8), dtype=torch.complex64, device="cuda")
    assert lib.fio3_apply(plan._h, f.data_ptr(), f.data_ptr(), None) == -1   # u aliases f
    with pytest.raises(ValueError):
        plan.apply(torch.zeros((8, 8, 4), dtype=torch.complex64, device="cuda"))


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-5)])
@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_3d_adjoint_identity(case, dtype, tol):
    """<v, B f> = <B^H v, f> with the forward that the oracle pins above: the
    adjoint is the exact conjugate transpose of every step."""
    import paper_0809_0719_amd as fio
    N, q, kind, s, lm = case
    plan = fio.Plan3(N, q, kind, s=s, lm=lm, dtype=dtype)
    f = torch.as_tensor(_noise(N, 11)).to(dtype).cuda()
    v = torch.as_tensor(_noise(N, 12)).to(dtype).cuda()
    u = plan.apply(f)
    g = plan.adjoint(v)
    lhs = torch.vdot(v.flatten().to(torch.complex128), u.flatten().to(torch.complex128)).item()
    rhs = torch.vdot(g.flatten().to(torch.complex128), f.flatten().to(torch.complex128)).item()
    print(f"3-D adjoint {case} {dtype}: <v,Bf> {lhs:.6e} <B^H v,f> {rhs:.6e}")
    assert abs(lhs - rhs) <= tol * abs(lhs)


def test_3d_adjoint_is_the_oracle_transpose():
    """N = 4, q = 5, eq:ex3, FP64: the dense matrix of the oracle's 3-D
    butterfly (its applies to the 64 unit inputs) transposed and conjugated,
    applied to v, against the library's adjoint."""
    import paper_0809_0719_amd as fio
    N, q = 4, 5
    model = B.ButterflyModel3(N, q, B.SPHERES)
    n3 = N ** 3
    Bm = np.empty((n3, n3), dtype=np.complex128)
    for j in range(n3):
        e = np.zeros(n3, dtype=np.complex128)
        e[j] = 1.0
        Bm[:, j] = model.apply(e.reshape(N, N, N)).ravel()
    v = _noise(N, 13)
    ref = (Bm.conj().T @ v.ravel()).reshape(N, N, N)
    plan = fio.Plan3(N, q, fio.SPHERES, dtype=torch.complex128)
    got = plan.adjoint(torch.as_tensor(v).cuda()).cpu().numpy()
    e = rel_max(got, ref)
    print(f"3-D adjoint vs dense oracle transpose: {e:.2e}")
    assert e <= 1e-12


def test_3d_autograd_backward_is_the_adjoint():
    """L = ||B f - y||^2 through FIOApply3: dL/d conj(f) = B^H (B f - y), the
    conjugate-Wirtinger gradient torch uses, equals 2 B^H(Bf - y) in torch's
    convention for real losses."""
    import paper_0809_0719_amd as fio
    N, q = 8, 5
    plan = fio.Plan3(N, q, fio.SPHERES, dtype=torch.complex128)
    f = torch.as_tensor(_noise(N, 14)).cuda().requires_grad_(True)
    y = torch.as_tensor(_noise(N, 15)).cuda()
    loss = (fio.FIOApply3.apply(f, plan) - y).abs().pow(2).sum()
    loss.backward()
    ref = 2 * plan.adjoint(plan.apply(f.detach()) - y)
    assert rel_l2(f.grad.cpu().numpy(), ref.cpu().numpy()) <= 1e-12
