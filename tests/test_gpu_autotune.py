"""The launch-shape autotuner (fio_plan_autotune, fio_plan_set_shape).

Every shape it chooses among runs the same arithmetic on each right-hand
side, so applies must be bit-identical across shapes; the forward result is
also checked against the FP64 oracle model for one right-hand side."""
import numpy as np
import pytest
import torch

from oracle import direct as D
from oracle.butterfly import ButterflyModel
from workloads import white_noise

from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu


def _dev(x, dtype=torch.complex64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


def test_every_shape_gives_the_same_results():
    import paper_0809_0719_amd as fio
    N, q, R = 256, 9, 64
    plan = fio.Plan(N, q, fio.Phase(), nrhs_max=R)
    assert plan.shape() == {"chunk": R, "switch_items": 16}
    F = _dev(white_noise(N, 5, nrhs=R))
    V = _dev(white_noise(N, 6, nrhs=R))
    U0, G0 = plan.apply(F), plan.adjoint(V)
    for chunk in (32, 64):
        for items in (8, 16, 32):
            plan.set_shape(chunk, items)
            assert plan.shape() == {"chunk": chunk, "switch_items": items}
            assert torch.equal(plan.apply(F), U0), (chunk, items)
            assert torch.equal(plan.adjoint(V), G0), (chunk, items)
    u_ref = ButterflyModel(N, q, D.Phase()).apply(white_noise(N, 5, nrhs=R)[7])
    assert rel_l2(U0[7].cpu().numpy(), u_ref) <= 2e-5


def test_autotune_keeps_a_measured_shape():
    import paper_0809_0719_amd as fio
    N, q, R = 256, 9, 64
    plan = fio.Plan(N, q, fio.Phase(), nrhs_max=R)
    F = _dev(white_noise(N, 8, nrhs=R))
    U0 = plan.apply(F)
    t = plan.autotune(R)
    print("autotune:", t)
    assert t["candidates"] == 6
    assert t["chunk"] in (32, 64) and t["switch_items"] in (8, 16, 32)
    assert plan.shape() == {"chunk": t["chunk"], "switch_items": t["switch_items"]}
    assert 0 < t["best_ms"] <= t["default_ms"]
    assert torch.equal(plan.apply(F), U0)


def test_autotune_leaves_untunable_plans_alone():
    import paper_0809_0719_amd as fio
    p64 = fio.Plan(64, 9, fio.Phase(), dtype=torch.complex128, nrhs_max=64)
    t = p64.autotune(64)
    assert t["candidates"] == 0 and p64.shape() == {"chunk": 64, "switch_items": 16}
    p1 = fio.Plan(64, 9, fio.Phase())
    assert p1.autotune(8)["candidates"] == 0
    # 48 right-hand sides: a chunk of 32 would leave 16 for a narrower pass
    p48 = fio.Plan(64, 9, fio.Phase(), nrhs_max=64)
    t = p48.autotune(48)
    assert t["candidates"] == 3 and t["chunk"] == 48
    with pytest.raises(RuntimeError):
        p48.set_shape(65, 16)
    with pytest.raises(RuntimeError):
        p48.set_shape(32, 12)
