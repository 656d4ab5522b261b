"""The matrix-core levels (contract="mfma"): chunks of 32 or more complex64
right-hand sides at q <= 9 run the p-levels and the adjoint x-levels as v_mfma_f32_4x4x1f32
contractions with the Chebyshev-symmetric halves of the interpolation
matrices, their inputs staged through LDS right-hand side innermost.

Checked against the single-right-hand-side applies of the same plan (the
vector-ALU kernels) to FP32 rounding, and one right-hand side of each batch
against the FP64 oracle model -- for every q the path serves, schedules with
p-levels and x-levels (N = 256: levels 4 and 5; N = 512: 4 and 5, 6) and
without (N = 128: x-level 4 only), batches that fill their 32-wide groups
partially (40), exactly (64), and spill into a second chunk that takes the
vector path (70 = 64 + 6)."""
import numpy as np
import pytest
import torch

from oracle import direct as D
from oracle.butterfly import ButterflyModel
from workloads import white_noise

from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

FP32_TOL = 2e-5


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).to(torch.complex64).cuda()


def _check(N, q, nr, nrhs_max, ph, seed):
    import paper_0809_0719_amd as fio
    phase = fio.Phase(ph.kind, ph.a1, ph.a2, ph.eta1, ph.eta2)
    one = fio.Plan(N, q, phase, dtype=torch.complex64)
    many = fio.Plan(N, q, phase, dtype=torch.complex64, nrhs_max=nrhs_max, contract="mfma")
    f = white_noise(N, seed, nrhs=nr)
    v = white_noise(N, seed + 1, nrhs=nr)
    F, V = _dev(f), _dev(v)
    print(f"levels_mm N={N} q={q} nr={nr} nrhs_max={nrhs_max}", flush=True)
    U = many.apply(F)
    G = many.adjoint(V)
    worst = 0.0
    for r in sorted({0, 1, 31, nr // 2, nr - 1} & set(range(nr))):
        e1 = rel_l2(U[r].cpu().numpy(), one.apply(F[r]).cpu().numpy())
        e2 = rel_l2(G[r].cpu().numpy(), one.adjoint(V[r]).cpu().numpy())
        worst = max(worst, e1, e2)
        assert e1 <= 2e-6 and e2 <= 2e-6, (r, e1, e2)
    r = nr - 1 if nr <= nrhs_max else nrhs_max - 1   # a right-hand side of the matrix-core chunk
    m = ButterflyModel(N, q, ph)
    eu = rel_l2(U[r].cpu().numpy(), m.apply(f[r]))
    eg = rel_l2(G[r].cpu().numpy(), m.adjoint(v[r]))
    print(f"  vs single applies {worst:.2e}; rhs {r} vs oracle: forward {eu:.2e}, adjoint {eg:.2e}")
    assert eu <= FP32_TOL and eg <= FP32_TOL


@pytest.mark.parametrize("q", [3, 4, 5, 6, 7, 8, 9])
def test_matrix_core_levels_every_q(q):
    _check(256, q, 40, 40, D.Phase(a1=1.05, a2=0.9, eta1=0.2, eta2=0.1), 100 + q)


@pytest.mark.parametrize("N,q,nr,nrhs_max", [(128, 9, 64, 64), (512, 7, 70, 64), (256, 9, 32, 32)])
def test_matrix_core_levels_schedules(N, q, nr, nrhs_max):
    _check(N, q, nr, nrhs_max, D.Phase(), 200 + N + q)


def test_matrix_core_levels_fourier_closed_form():
    """The Fourier phase at N = 256, q = 9 through the matrix-core path against
    the closed form N^2 IDFT(ifftshift(f)) (the butterfly's own error for this
    phase is ~2e-2 at q = 9, N = 256) and against the single applies."""
    import paper_0809_0719_amd as fio
    N, q, nr = 256, 9, 32
    f = white_noise(N, 7, nrhs=nr)
    plan = fio.Plan(N, q, fio.Phase(kind=fio.FOURIER), dtype=torch.complex64, nrhs_max=nr, contract="mfma")
    U = plan.apply(_dev(f)).cpu().numpy()
    for r in (0, nr - 1):
        ref = N * N * np.fft.ifft2(np.fft.ifftshift(f[r]))
        e = rel_l2(U[r], ref)
        print(f"Fourier N={N} q={q} rhs {r} vs closed form: {e:.2e}")
        assert e < 5e-2


def test_matrix_core_levels_plan_limits():
    import paper_0809_0719_amd as fio
    with pytest.raises(RuntimeError):
        fio.Plan(64, 10, contract="mfma")
    with pytest.raises(RuntimeError):
        fio.Plan(64, 9, dtype=torch.complex128, contract="mfma")
    with pytest.raises(ValueError):
        fio.Plan(64, 9, contract="tf32")
