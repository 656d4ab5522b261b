"""BF16 contractions on the matrix cores (contract="bf16"): parity with the
FP64 oracle within the BF16 rounding budget.

Tolerance: every BF16 level rounds the operands of its two 1-D passes to
8 significant bits (relative error <= 2^-9 per operand, ~2^-9/sqrt(3) rms);
a pass sums 2q such terms with FP32 accumulation, so each level adds about
1e-3 relative rms error; BF16_TOL covers the levels of the cases below with
a 3x margin."""
import numpy as np
import pytest
import torch

from oracle import direct as D
from oracle.butterfly import ButterflyModel
from workloads import white_noise

from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

BF16_TOL = 1e-2


def _dev(x, dtype=torch.complex64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


@pytest.mark.parametrize("N,q,s,nrhs", [(32, 7, 1, 20), (64, 9, 2, 17), (256, 7, None, 16), (64, 5, 1, 3)])
def test_bf16_contractions_match_oracle(N, q, s, nrhs):
    import paper_0809_0719_amd as fio
    plan = fio.Plan(N, q, fio.Phase(), s=s, nrhs_max=nrhs, contract="bf16")
    F = np.stack([white_noise(N, 50 + r) for r in range(nrhs)])
    U = plan.apply(_dev(F)).cpu().numpy()
    m = ButterflyModel(N, q, D.Phase(), s=s)
    worst = 0.0
    for r in (0, nrhs // 2, nrhs - 1):
        e = rel_l2(U[r], m.apply(F[r]))
        worst = max(worst, e)
    print(f"bf16 N={N} q={q} s={s} nrhs={nrhs}: worst rel_l2 vs oracle {worst:.2e}")
    assert worst <= BF16_TOL


def test_bf16_rejects_unsupported_configurations():
    import paper_0809_0719_amd as fio
    with pytest.raises(RuntimeError):
        fio.Plan(64, 13, contract="bf16")
    with pytest.raises(RuntimeError):
        fio.Plan(64, 9, dtype=torch.complex128, contract="bf16")
