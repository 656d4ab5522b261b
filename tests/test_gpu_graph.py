"""Graph capture of the butterfly: a plan's forward and adjoint launches go to
the caller's stream and allocate nothing, so they can be captured in a HIP
graph (through torch.cuda.graph) and replayed.  Every replay is checked
against an eager apply of the same inputs, with eager work and
synchronisations between the replays."""
import numpy as np
import pytest
import torch

from workloads import white_noise

from gpu_helpers import rel_max

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,q,nrhs", [(64, 5, 2), (32, 7, 1)])
def test_captured_apply_and_adjoint_replay(N, q, nrhs):
    import paper_0809_0719_amd as fio
    plan = fio.Plan(N, q, fio.Phase(a1=1.05, a2=0.97), nrhs_max=nrhs)
    shape = (nrhs, N, N)
    f_static = torch.zeros(shape, dtype=torch.complex64, device="cuda")
    g_static = torch.zeros(shape, dtype=torch.complex64, device="cuda")
    # warm-up on a side stream (tables made, kernels loaded) before capture
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.apply(f_static)
        plan.adjoint(g_static)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        u_static = plan.apply(f_static)
        h_static = plan.adjoint(g_static)

    for rep in range(3):
        f = torch.as_tensor(white_noise(N, 60 + rep, nrhs=nrhs).reshape(shape)).to(torch.complex64).cuda()
        g = torch.as_tensor(white_noise(N, 70 + rep, nrhs=nrhs).reshape(shape)).to(torch.complex64).cuda()
        f_static.copy_(f)
        g_static.copy_(g)
        graph.replay()
        torch.cuda.synchronize()
        u_eager = plan.apply(f)
        h_eager = plan.adjoint(g)
        torch.cuda.synchronize()
        e1 = rel_max(u_static.cpu().numpy(), u_eager.cpu().numpy())
        e2 = rel_max(h_static.cpu().numpy(), h_eager.cpu().numpy())
        print(f"replay {rep}: forward {e1:.1e}, adjoint {e2:.1e}")
        assert e1 == 0.0 and e2 == 0.0, (rep, e1, e2)
        # unrelated eager work between replays
        _ = (f * 2).sum().item()
