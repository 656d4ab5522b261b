"""Parity of the HIP butterfly (through the C ABI) with the FP64 oracle.

Tolerances (relative, over all outputs of a case):
* FP64 path (complex128): 1e-10.  Both sides compute the same formulas in
  FP64; the differences are rounding order and the factorised phase
  rho(p1) * Phi(x, e(theta)) vs. Phi(x, k(p)), ~1e-13 cycles on phases of
  ~N cycles, amplified by the O(1) Lebesgue constants of the levels.
* FP32 path (complex64): see FP32_TOL; the exponentials of the FP64-reduced
  phases are taken in FP32 (abs. error ~1e-6) and the contractions round to
  FP32 (2^-24 per operation, ~q terms per pass), accumulated over the
  2 + levels steps of the pass.
"""
import functools

import numpy as np
import pytest
import torch

from oracle import direct as D
from oracle.butterfly import ButterflyModel
from workloads import white_noise

from gpu_helpers import rel_l2, rel_max, weights_to_oracle

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 2e-5

# (N, q, phase, s, lm)
CASES = [
    (8, 5, D.Phase(), None, None),                        # smallest N: s=1, lm=1
    (16, 3, D.Phase(), None, None),                       # smallest q, no recursion levels
    (32, 5, D.Phase(), None, None),                       # C0 geometry (L odd, s=2, lm=2)
    (32, 7, D.Phase(kind=D.FOURIER), 1, 2),               # p-level 2, x-levels 3, 4
    (32, 6, D.Phase(a1=1.1, a2=0.9, eta1=0.2, eta2=0.1), 1, 3),  # even q, other switch level
    (64, 9, D.Phase(), 2, None),                          # p-level 3, x-level 4
    (64, 5, D.Phase(), 0, None),                          # s = 0: Sec. 4 verbatim
    (128, 7, D.Phase(a1=0.85, a2=1.15), None, None),      # L odd, x-level 4
    (16, 16, D.Phase(), None, None),                      # largest q
]


def _ids(c):
    N, q, ph, s, lm = c
    return f"N{N}-q{q}-k{ph.kind}-s{s}-lm{lm}"


@functools.lru_cache(maxsize=None)
def oracle_forward(N, q, ph, s, lm, seed):
    m = ButterflyModel(N, q, ph, s=s, lm=lm)
    u, lev = m.apply(white_noise(N, seed), return_levels=True)
    return m, u, lev


@functools.lru_cache(maxsize=None)
def oracle_adjoint(N, q, ph, s, lm, seed):
    m = ButterflyModel(N, q, ph, s=s, lm=lm)
    return m.adjoint(white_noise(N, seed))


def _plan(N, q, ph, s, lm, dtype):
    import paper_0809_0719_amd as fio
    return fio.Plan(N, q, fio.Phase(ph.kind, ph.a1, ph.a2, ph.eta1, ph.eta2), s=s, lm=lm, dtype=dtype)


def _dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_forward_parity_fp64(case):
    N, q, ph, s, lm = case
    _, u_ref, _ = oracle_forward(N, q, ph, s, lm, 1)
    plan = _plan(N, q, ph, s, lm, torch.complex128)
    u = plan.apply(_dev(white_noise(N, 1), torch.complex128)).cpu().numpy()
    e2, em = rel_l2(u, u_ref), rel_max(u, u_ref)
    print(f"forward fp64 {case}: rel_l2 {e2:.2e} rel_max {em:.2e}")
    assert e2 <= FP64_TOL and em <= FP64_TOL


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_forward_parity_fp32(case):
    N, q, ph, s, lm = case
    _, u_ref, _ = oracle_forward(N, q, ph, s, lm, 1)
    plan = _plan(N, q, ph, s, lm, torch.complex64)
    u = plan.apply(_dev(white_noise(N, 1), torch.complex64)).cpu().numpy()
    e2, em = rel_l2(u, u_ref), rel_max(u, u_ref)
    print(f"forward fp32 {case}: rel_l2 {e2:.2e} rel_max {em:.2e}")
    assert e2 <= FP32_TOL and em <= 4 * FP32_TOL


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_adjoint_parity_fp64(case):
    N, q, ph, s, lm = case
    f_ref = oracle_adjoint(N, q, ph, s, lm, 2)
    plan = _plan(N, q, ph, s, lm, torch.complex128)
    f = plan.adjoint(_dev(white_noise(N, 2), torch.complex128)).cpu().numpy()
    e2, em = rel_l2(f, f_ref), rel_max(f, f_ref)
    print(f"adjoint fp64 {case}: rel_l2 {e2:.2e} rel_max {em:.2e}")
    assert e2 <= FP64_TOL and em <= FP64_TOL


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_adjoint_parity_fp32(case):
    N, q, ph, s, lm = case
    f_ref = oracle_adjoint(N, q, ph, s, lm, 2)
    plan = _plan(N, q, ph, s, lm, torch.complex64)
    f = plan.adjoint(_dev(white_noise(N, 2), torch.complex64)).cpu().numpy()
    e2, em = rel_l2(f, f_ref), rel_max(f, f_ref)
    print(f"adjoint fp32 {case}: rel_l2 {e2:.2e} rel_max {em:.2e}")
    assert e2 <= FP32_TOL and em <= 4 * FP32_TOL


@pytest.mark.parametrize("case", [CASES[3], CASES[5], CASES[7]], ids=_ids)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_every_stage_matches_the_oracle(case, dtype):
    N, q, ph, s, lm = case
    m, _, lev = oracle_forward(N, q, ph, s, lm, 1)
    keys = ["init"] + [("p", l) for l in range(m.s + 1, m.lm + 1)] + ["switch"] + \
           [("x", l) for l in range(m.lm + 1, m.L - m.s + 1)]
    plan = _plan(N, q, ph, s, lm, dtype)
    assert plan.n_stages == len(keys)
    f = _dev(white_noise(N, 1), dtype)
    tol = FP64_TOL if dtype == torch.complex128 else FP32_TOL
    for st, key in enumerate(keys):
        w = weights_to_oracle(plan.debug_stage(f, st).cpu().numpy(), N, q, plan.stage_level(st))
        e2 = rel_l2(w, lev[key])
        print(f"stage {st} {key}: rel_l2 {e2:.2e}")
        assert e2 <= tol, (st, key, e2)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_dot_product_identity_and_linearity(dtype):
    N, q = 64, 7
    plan = _plan(N, q, D.Phase(), None, None, dtype)
    f = _dev(white_noise(N, 3), dtype)
    g = _dev(white_noise(N, 4), dtype)
    u = _dev(white_noise(N, 5), dtype)
    Bf = plan.apply(f)
    lhs = torch.vdot(u.flatten(), Bf.flatten()).item()
    rhs = torch.vdot(plan.adjoint(u).flatten(), f.flatten()).item()
    tol = 1e-12 if dtype == torch.complex128 else 1e-5
    assert abs(lhs - rhs) <= tol * abs(lhs)
    a, b = 0.5 - 1.5j, 2.0 + 0.25j
    lin = plan.apply(a * f + b * g) - (a * Bf + b * plan.apply(g))
    assert lin.abs().max().item() <= (1e-12 if dtype == torch.complex128 else 1e-5) * Bf.abs().max().item()


def test_several_right_hand_sides_and_zero_input():
    N, q = 32, 5
    plan = _plan(N, q, D.Phase(), None, None, torch.complex64)
    F = np.stack([white_noise(N, 10 + r) for r in range(3)])
    U = plan.apply(_dev(F, torch.complex64)).cpu().numpy()
    for r in range(3):
        one = plan.apply(_dev(F[r], torch.complex64)).cpu().numpy()
        assert np.array_equal(U[r], one)          # same kernels, same inputs: bit-identical
    z = plan.apply(torch.zeros(N, N, dtype=torch.complex64, device="cuda"))
    assert z.abs().max().item() == 0.0


def test_deterministic():
    N, q = 64, 9
    plan = _plan(N, q, D.Phase(), None, None, torch.complex64)
    f = _dev(white_noise(N, 6), torch.complex64)
    assert torch.equal(plan.apply(f), plan.apply(f))
    assert torch.equal(plan.adjoint(f), plan.adjoint(f))


def test_fourier_phase_approximates_fft():
    # the butterfly with Phi = x.k approximates N^2 * IDFT(ifftshift(f)); its
    # error equals the oracle model's (parity) and shrinks with q
    N = 64
    f = white_noise(N, 7)
    ref = N * N * np.fft.ifft2(np.fft.ifftshift(f))
    errs = []
    for q in (9, 13):
        plan = _plan(N, q, D.Phase(kind=D.FOURIER), 2, None, torch.complex128)
        u = plan.apply(_dev(f, torch.complex128)).cpu().numpy()
        errs.append(rel_l2(u, ref))
    assert errs[1] < errs[0] / 10


def test_bad_arguments_raise():
    import paper_0809_0719_amd as fio
    with pytest.raises(RuntimeError):
        fio.Plan(48, 9)
    with pytest.raises(RuntimeError):
        fio.Plan(64, 9, s=4)
    plan = fio.Plan(32, 5)
    with pytest.raises(TypeError):
        plan.apply(torch.zeros(32, 32, dtype=torch.complex128, device="cuda"))
    with pytest.raises(ValueError):
        plan.apply(torch.zeros(16, 16, dtype=torch.complex64, device="cuda"))
    with pytest.raises(RuntimeError):
        plan.debug_stage(torch.zeros(32, 32, dtype=torch.complex64, device="cuda"), 99)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_full_size_sampled_parity(dtype):
    """The benchmark's configuration (N=1024, q=9, eq:ex1, s=3, lm=5): the
    oracle computes the ancestor chains of a few sampled leaf boxes A (level
    L-s) and the GPU must match it on those boxes' 64 potentials each and on
    every stage's weights of those ancestors."""
    N, q = 1024, 9
    rng = np.random.default_rng(2024)
    targets = [tuple(int(v) for v in rng.integers(0, 128, 2)) for _ in range(2)]
    m = ButterflyModel(N, q, D.Phase())
    f = white_noise(N, 21)
    u_ref, lev = m.apply(f, return_levels=True, targets=targets)
    plan = _plan(N, q, D.Phase(), None, None, dtype)
    fd = _dev(f, dtype)
    u = plan.apply(fd).cpu().numpy()
    tol = FP64_TOL if dtype == torch.complex128 else FP32_TOL
    side = 1 << m.s
    got, ref = [], []
    for a1, a2 in targets:
        blk = (slice(a1 * side, (a1 + 1) * side), slice(a2 * side, (a2 + 1) * side))
        got.append(u[blk])
        ref.append(u_ref[blk])
    e2 = rel_l2(np.array(got), np.array(ref))
    print(f"full size {dtype}: potentials rel_l2 {e2:.2e}")
    assert e2 <= tol
    keys = ["init"] + [("p", l) for l in range(m.s + 1, m.lm + 1)] + ["switch"] + \
           [("x", l) for l in range(m.lm + 1, m.L - m.s + 1)]
    for st, key in enumerate(keys):
        level = plan.stage_level(st)
        w = plan.debug_stage(fd, st).cpu().numpy().reshape(N * N, q, q)
        nB = 1 << (m.L - level)
        from gpu_helpers import morton
        bm = morton(*np.meshgrid(np.arange(nB), np.arange(nB), indexing="ij"))
        for (a1, a2), wref in lev[key].items():
            pair = int(morton(a1, a2)) * nB * nB + bm
            e = rel_l2(w[pair], wref)
            assert e <= tol, (st, key, (a1, a2), e)
        print(f"  stage {st} {key}: ok")
        del w


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("case", [CASES[3], CASES[5], (32, 16, D.Phase(), 1, None)], ids=_ids)
def test_batched_equals_one_by_one(case, dtype):
    """nrhs_max right-hand sides share every kernel value of the levels and
    the switch (7 = 5 + 2: a full and a ragged chunk).  The batched kernels
    compute the same formulas as the single-RHS ones with the exponentials
    hoisted out of the right-hand-side loop, so they agree to rounding:
    a few ulps per operation of the pass."""
    N, q, ph, s, lm = case
    import paper_0809_0719_amd as fio
    phase = fio.Phase(ph.kind, ph.a1, ph.a2, ph.eta1, ph.eta2)
    one = fio.Plan(N, q, phase, s=s, lm=lm, dtype=dtype)
    many = fio.Plan(N, q, phase, s=s, lm=lm, dtype=dtype, nrhs_max=5)
    F = _dev(np.stack([white_noise(N, 30 + r) for r in range(7)]), dtype)
    U = many.apply(F)
    G = many.adjoint(U)
    tol = 1e-13 if dtype == torch.complex128 else 2e-6
    for r in range(7):
        e1 = rel_l2(U[r].cpu().numpy(), one.apply(F[r]).cpu().numpy())
        e2 = rel_l2(G[r].cpu().numpy(), one.adjoint(U[r]).cpu().numpy())
        assert e1 <= tol and e2 <= tol, (r, e1, e2)
    # and one right-hand side of the batch against the oracle directly
    if case[0] <= 64:
        _, u_ref, _ = oracle_forward(N, q, ph, s, lm, 36)
        assert rel_l2(U[6].cpu().numpy(), u_ref) <= (FP64_TOL if dtype == torch.complex128 else FP32_TOL)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_batched_termination_more_than_64_rhs(dtype):
    """70 right-hand sides: the one-lane-per-RHS termination kernels take
    them in two groups of 64 lanes, the second ragged.  Against one-at-a-time
    applies (N = 64, s = 3: 8 grid columns over 5 waves)."""
    import paper_0809_0719_amd as fio
    N, q = 64, 5
    one = fio.Plan(N, q, fio.Phase(), dtype=dtype)
    many = fio.Plan(N, q, fio.Phase(), dtype=dtype, nrhs_max=70)
    F = _dev(white_noise(N, 50, nrhs=70), dtype)
    U = many.apply(F)
    G = many.adjoint(U)
    tol = 1e-13 if dtype == torch.complex128 else 2e-6
    for r in (0, 1, 63, 64, 69):
        e1 = rel_l2(U[r].cpu().numpy(), one.apply(F[r]).cpu().numpy())
        e2 = rel_l2(G[r].cpu().numpy(), one.adjoint(U[r]).cpu().numpy())
        assert e1 <= tol and e2 <= tol, (r, e1, e2)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("N,q,s", [(64, 9, 3), (32, 5, 2), (32, 3, 1), (16, 4, 0), (64, 12, 3), (64, 8, 3)])
def test_wide_batched_termination(N, q, s, dtype):
    """Batches of 32 or more right-hand sides take the one-lane-per-RHS
    termination kernels where they fit (complex64 q <= 12, complex128
    q <= 8; the others keep the 16-per-wave kernels): 40 right-hand sides
    leave 24 lanes idle.  Every s from 0 to 3 (2^s grid columns, fewer or
    more than the q waves).  Against one-at-a-time applies, and one
    right-hand side against the oracle."""
    import paper_0809_0719_amd as fio
    nr = 40
    ph = D.Phase(a1=1.1, a2=0.95)
    phase = fio.Phase(ph.kind, ph.a1, ph.a2)
    one = fio.Plan(N, q, phase, s=s, dtype=dtype)
    many = fio.Plan(N, q, phase, s=s, dtype=dtype, nrhs_max=nr)
    F = _dev(white_noise(N, 80, nrhs=nr), dtype)
    U = many.apply(F)
    G = many.adjoint(U)
    tol = 1e-13 if dtype == torch.complex128 else 2e-6
    for r in (0, 17, 39):
        e1 = rel_l2(U[r].cpu().numpy(), one.apply(F[r]).cpu().numpy())
        e2 = rel_l2(G[r].cpu().numpy(), one.adjoint(U[r]).cpu().numpy())
        assert e1 <= tol and e2 <= tol, (r, e1, e2)
    f39 = white_noise(N, 80, nrhs=nr)[39]
    u_ref = ButterflyModel(N, q, ph, s=s).apply(f39)
    e = rel_l2(U[39].cpu().numpy(), u_ref)
    print(f"wide termination N={N} q={q} s={s} {dtype}: rhs 39 vs oracle {e:.2e}")
    assert e <= (FP64_TOL if dtype == torch.complex128 else FP32_TOL)


def test_grid_beyond_2_32_work_items():
    """N = 4096, q = 12: the switch has one pair per workgroup, 2^24
    workgroups of 256 threads -- 2^32 work-items, past the limit of one grid
    dimension, so the launch spreads the workgroups over two.  Checked with
    the Fourier phase against the closed form N^2 IDFT(ifftshift(f)); the
    oracle model's error at q = 12 is 7.9e-4 (N = 64) and 9.5e-4 (N = 128),
    slowly growing with N."""
    import paper_0809_0719_amd as fio
    N, q = 4096, 12
    f = white_noise(N, 9)
    ref = N * N * np.fft.ifft2(np.fft.ifftshift(f))
    plan = fio.Plan(N, q, fio.Phase(kind=fio.FOURIER))
    u = plan.apply(_dev(f, torch.complex64)).cpu().numpy()
    del plan
    e = rel_l2(u, ref)
    print(f"N={N} q={q} Fourier phase vs closed form: {e:.2e}")
    assert e < 5e-3


def test_full_size_batched_parity_in_the_benchmark_configuration():
    """N = 1024, q = 9, eq:ex1, complex64, nrhs_max = 64 and 64 right-hand
    sides (the inputs the benchmark times, white noise seed 3): the batched
    kernels (matrix-core initialisation for two right-hand sides per pass,
    hoisted levels, the switch and its adjoint on the matrix cores,
    one-lane-per-RHS termination)
    against the oracle's restricted pass on two sampled leaf boxes for the
    first and the last right-hand side; and the batched adjoint through the
    identity sum_r <v_r, B f_r> = sum_r <B^H v_r, f_r>, which holds at any
    size (FP32 path: relative 1e-4)."""
    import paper_0809_0719_amd as fio
    N, q, R = 1024, 9, 64
    f = white_noise(N, 3, nrhs=R)
    plan = fio.Plan(N, q, fio.Phase(), dtype=torch.complex64, nrhs_max=R)
    fd = _dev(f, torch.complex64)
    u = plan.apply(fd)
    rng = np.random.default_rng(77)
    targets = [tuple(int(v) for v in rng.integers(0, 128, 2)) for _ in range(2)]
    side = 8
    for r in (0, R - 1):
        u_ref = ButterflyModel(N, q, D.Phase()).apply(f[r], targets=targets)
        ur = u[r].cpu().numpy()
        got = np.array([ur[a1 * side:(a1 + 1) * side, a2 * side:(a2 + 1) * side] for a1, a2 in targets])
        ref = np.array([u_ref[a1 * side:(a1 + 1) * side, a2 * side:(a2 + 1) * side] for a1, a2 in targets])
        e = rel_l2(got, ref)
        print(f"batched full size, rhs {r}: {e:.2e}")
        assert e <= FP32_TOL
    v = _dev(white_noise(N, 4, nrhs=R), torch.complex64)
    g = plan.adjoint(v)
    lhs = torch.vdot(v.flatten().to(torch.complex128), u.flatten().to(torch.complex128)).item()
    rhs = torch.vdot(g.flatten().to(torch.complex128), fd.flatten().to(torch.complex128)).item()
    print(f"<v, B f> = {lhs:.6e}, <B^H v, f> = {rhs:.6e}")
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


def test_full_size_batched_adjoint_parity_in_the_benchmark_configuration():
    """The batched adjoint in the benchmark's configuration (N = 1024, q = 9,
    eq:ex1, complex64, 64 right-hand sides: the wide termination^H, the
    adjoint levels, the matrix-core switch^H and initialisation^H) against
    the oracle's adjoint restricted to three sampled source boxes at level
    L - s of T_P, element by element at every source inside them, for the
    first and the last right-hand side."""
    import paper_0809_0719_amd as fio
    from oracle.butterfly import box_of
    N, q, R = 1024, 9, 64
    v = white_noise(N, 4, nrhs=R)
    plan = fio.Plan(N, q, fio.Phase(), dtype=torch.complex64, nrhs_max=R)
    print(f"adjoint N={N} q={q} nrhs={R}", flush=True)
    g = plan.adjoint(_dev(v, torch.complex64))
    model = ButterflyModel(N, q, D.Phase())
    lB = model.L - model.s
    b1, b2 = box_of(model.p1, lB), box_of(model.p2, lB)
    pick = np.random.default_rng(78).choice(N * N, 3, replace=False)   # boxes of three sampled sources
    sources = sorted({(int(b1[j]), int(b2[j])) for j in pick})
    mask = np.zeros(N * N, dtype=bool)
    for c1, c2 in sources:
        mask |= (b1 == c1) & (b2 == c2)
    for r in (0, R - 1):
        f_ref = model.adjoint(v[r], sources=sources).ravel()[mask]
        got = g[r].cpu().numpy().ravel()[mask]
        e, em = rel_l2(got, f_ref), rel_max(got, f_ref)
        print(f"batched adjoint full size, rhs {r}, {mask.sum()} sources: rel l2 {e:.2e}, rel max {em:.2e}")
        assert e <= FP32_TOL and em <= 4 * FP32_TOL


@pytest.mark.parametrize("nr", [33, 65])
@pytest.mark.parametrize("q", [3, 4, 5, 6, 7, 8, 9])
def test_matrix_core_switch(q, nr):
    """The forward switch of batches of 32 or more complex64 right-hand sides
    at q <= 9 on the matrix cores, against the single-RHS forward (vector
    switch), as for the adjoint below."""
    import paper_0809_0719_amd as fio
    N = 32
    one = fio.Plan(N, q, fio.Phase(), dtype=torch.complex64)
    many = fio.Plan(N, q, fio.Phase(), dtype=torch.complex64, nrhs_max=nr)
    F = _dev(white_noise(N, 90 + q, nrhs=nr), torch.complex64)
    U = many.apply(F)
    for r in (0, 17, 32, nr - 1):
        e = rel_l2(U[r].cpu().numpy(), one.apply(F[r]).cpu().numpy())
        assert e <= 2e-6, (r, e)


@pytest.mark.parametrize("nr", [33, 65])
@pytest.mark.parametrize("q", [3, 4, 5, 6, 7, 8, 9])
def test_matrix_core_adjoint_switch(q, nr):
    """Batches of 32 or more complex64 right-hand sides at q <= 9 take the
    adjoint switch on the matrix cores (chunks of 64: 33 leaves 31 columns
    empty, 65 adds a second chunk of one); the single-RHS adjoint keeps the
    vector kernel.  The two agree to rounding on every right-hand side
    checked, for odd and even q (the odd q add the middle row s1 = q//2)."""
    import paper_0809_0719_amd as fio
    N = 32
    one = fio.Plan(N, q, fio.Phase(), dtype=torch.complex64)
    many = fio.Plan(N, q, fio.Phase(), dtype=torch.complex64, nrhs_max=nr)
    V = _dev(white_noise(N, 70 + q, nrhs=nr), torch.complex64)
    G = many.adjoint(V)
    for r in (0, 17, 32, nr - 1):
        e = rel_l2(G[r].cpu().numpy(), one.adjoint(V[r]).cpu().numpy())
        assert e <= 2e-6, (r, e)
