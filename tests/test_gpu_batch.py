"""Uneven batches of plans (fio_batch_*), the direct evaluation at sampled
targets (fio_direct_rows) and the choice of q by the estimated error eq:err
(fio_select_q).

* direct_rows is the definition eq:dfio; it is checked against the oracle's
  direct sum (C, FP64) at the same targets.
* select_q's probe and targets are SplitMix64 draws; the test side makes the
  same draws with its own implementation of the published generator
  (workloads) and recomputes every estimate with the FP64 oracle butterfly
  and the oracle's direct sum, so both the estimates and the choice are
  checked against the oracle.
* A batch runs each plan's own apply on an internal stream; its outputs are
  compared with the plans' individual applies bit for bit, also when the
  batch is replayed from a captured graph.
"""
import numpy as np
import pytest
import torch

from oracle import direct as D
from oracle.butterfly import ButterflyModel
from workloads import mixed_batch, probe_phases, probe_rows, white_noise

from gpu_helpers import rel_max

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


def _fphase(ph):
    import paper_0809_0719_amd as fio
    return fio.Phase(ph.kind, ph.a1, ph.a2, ph.eta1, ph.eta2)


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-6)])
@pytest.mark.parametrize("N,ph,nrows", [(32, D.Phase(a1=1.1, a2=0.9, eta1=0.2), None),
                                        (256, D.Phase(), 64),
                                        (128, D.Phase(kind=D.FOURIER), 40)])
def test_direct_rows_match_oracle(N, ph, nrows, dtype, tol):
    import paper_0809_0719_amd as fio
    plan = fio.Plan(N, 5, _fphase(ph), dtype=dtype)
    f = white_noise(N, 3)
    fd = _dev(f, dtype)
    rows = np.arange(N * N) if nrows is None else probe_rows(N, nrows, 11)
    out = fio.direct_rows(plan, fd, torch.as_tensor(rows)).cpu().numpy()
    # the oracle sees the same (rounded) input the library stores
    ref = D.forward(N, ph, fd.cpu().numpy().astype(np.complex128), rows)
    e = rel_max(out, ref)
    print(f"direct rows N={N} kind={ph.kind} {dtype}: {e:.2e}")
    assert e <= tol


@pytest.mark.parametrize("dtype,etol", [(torch.complex128, 1e-9), (torch.complex64, 2e-5)])
@pytest.mark.parametrize("ph,tol,want", [(D.Phase(kind=D.FOURIER), 0.05, 8), (D.Phase(), 0.6, 7)])
def test_select_q_matches_oracle_estimates(ph, tol, want, dtype, etol):
    """N = 32, probe seed 5, 64 targets.  Oracle estimates (FP64 butterfly vs
    the direct sum, eq:err): Fourier phase 0.068 at q = 7, 0.022 at q = 8;
    eq:ex1 0.70 at q = 6, 0.52 at q = 7, so the tolerances choose q = 8 and 7
    with margins on both sides."""
    import paper_0809_0719_amd as fio
    N, seed, nrows = 32, 5, 64
    q, err, tried = fio.select_q(N, _fphase(ph), tol=tol, qmin=3, qmax=12, nrows=nrows, seed=seed, dtype=dtype)
    f = probe_phases(N, seed)
    if dtype == torch.complex64:
        f = f.astype(np.complex64).astype(np.complex128)
    rows = probe_rows(N, nrows, seed)
    ref = D.forward(N, ph, f, rows)
    print(f"select_q kind={ph.kind} {dtype}: q={q} err={err:.4g} tried={ {k: round(v, 5) for k, v in tried.items()} }")
    for qq, e in tried.items():
        e_or = D.rel_err(ref, ButterflyModel(N, qq, ph).apply(f).ravel()[rows])
        assert abs(e - e_or) <= etol * max(1.0, e_or), (qq, e, e_or)
    assert q == want and sorted(tried) == list(range(3, want + 1))
    assert err == tried[q] and err <= tol and tried[q - 1] > tol


def test_select_q_reports_when_no_q_reaches_tol():
    import paper_0809_0719_amd as fio
    q, err, tried = fio.select_q(16, fio.Phase(), tol=1e-9, qmin=3, qmax=5, nrows=16, seed=1)
    assert q == 5 and err > 1e-9 and sorted(tried) == [3, 4, 5]


def _mixed_plans():
    """A mixed batch after the C4 recipe (N and eta from the seeded draw,
    N capped at 256 and q from {4,..,9} so the test stays small), plus two
    complex128 problems."""
    import paper_0809_0719_amd as fio
    probs = mixed_batch(6, n=6)
    plans, inputs = [], []
    for i, p in enumerate(probs):
        N = min(p["N"], 256) >> (i % 3)
        dtype = torch.complex128 if i % 3 == 2 else torch.complex64
        plan = fio.Plan(N, 4 + i, fio.Phase(eta1=p["eta1"], eta2=p["eta2"]), dtype=dtype)
        plans.append(plan)
        inputs.append(_dev(white_noise(N, p["f_seed"] % 1000), dtype))
    return plans, inputs


@pytest.mark.parametrize("nstreams", [1, 4])
def test_batch_equals_individual_applies(nstreams):
    import paper_0809_0719_amd as fio
    plans, fs = _mixed_plans()
    batch = fio.Batch(plans, nstreams=nstreams)
    us = batch.apply(fs)
    gs = batch.adjoint(us)
    torch.cuda.synchronize()
    for p, f, u, g in zip(plans, fs, us, gs):
        assert torch.equal(u, p.apply(f)), (p.N, p.q)
        assert torch.equal(g, p.adjoint(u)), (p.N, p.q)
    # one problem against the oracle as well
    p, f, u = plans[1], fs[1], us[1]
    ph = D.Phase(eta1=p.phase.eta1, eta2=p.phase.eta2)
    u_ref = ButterflyModel(p.N, p.q, ph).apply(f.cpu().numpy().astype(np.complex128))
    assert rel_max(u.cpu().numpy(), u_ref) <= 1e-4


def test_batch_graph_capture_replays():
    """A stream capture of the batch records the fork onto the internal
    streams and the join; replays with new inputs equal eager batch applies,
    with eager work between the replays."""
    import paper_0809_0719_amd as fio
    plans, fs = _mixed_plans()
    batch = fio.Batch(plans, nstreams=3)
    f_static = [torch.zeros_like(f) for f in fs]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.apply(f_static)  # tables made before the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        u_static = batch.apply(f_static)
    for rep in range(3):
        new = [_dev(white_noise(p.N, 90 + rep), p.dtype) for p in plans]
        for s, n in zip(f_static, new):
            s.copy_(n)
        graph.replay()
        torch.cuda.synchronize()
        eager = batch.apply(new)
        torch.cuda.synchronize()
        for a, b in zip(u_static, eager):
            assert torch.equal(a, b), rep
        _ = sum(float(x.abs().sum()) for x in new)


def test_batch_bad_arguments():
    import ctypes
    import paper_0809_0719_amd as fio
    p = fio.Plan(16, 4, fio.Phase())
    with pytest.raises(ValueError):
        fio.Batch([p, p])
    lib = fio.load_library()
    handles = (ctypes.c_void_p * 2)(p._h.value, p._h.value)
    h = ctypes.c_void_p()
    assert lib.fio_batch_create(handles, 2, 2, ctypes.byref(h)) == -1
    assert b"twice" in lib.fio_last_error()
    batch = fio.Batch([p])
    f = _dev(white_noise(16, 1), torch.complex64)
    with pytest.raises(ValueError):
        batch.apply([f, f])
    with pytest.raises(ValueError):
        batch.apply([f], outs=[f])  # output aliases the input: the binding refuses it
    a = (ctypes.c_void_p * 1)(f.data_ptr())
    assert lib.fio_batch_apply(batch._h, a, a, None) == -1          # and so does the library
    assert lib.fio_batch_apply_adjoint(batch._h, a, a, None) == -1
