"""Benchmark of the butterfly FIO pass on one MI355X.

Workload (eq:ex1 of the numerical section, constant amplitude): N = 1024,
q = 9 Chebyshev points per dimension, s = 3 (recursion from level L-3 of T_P
to level 3), switch at level 5; sources f are complex white noise, resident
in HBM before the timed region.  FP64 phases with their FP64 mod-1
reduction; FP32 weights and contractions.

One step = one forward apply u = B f and one adjoint apply g = B^H u of a
batch of `nrhs` right-hand sides: the whole pass (initialisation, p-levels,
switch, x-levels, termination) in both directions.  `value` counts every
forward and every adjoint application of one right-hand side as one apply.

Printed on one JSON line: throughput, the roofline of the dominant kernel
(its time measured with HIP events recorded on the launch stream inside the
timed region), the relative error eq:err against the FP64 direct sum on 256
sampled points, and the CPU baseline: the direct-sum oracle timed on the
host on 3072 sampled points (about 10 s) and extrapolated to all N^2 points.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FIO applies/sec at N=1024,q=9, rel err ≤1e-4; batched+adjoint vs plain"

# MI355X peaks
HBM_PEAK_GBS = 8000.0
# VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations/s
# (an FP32 or FP64 FMA is one lane-op; sine, cosine, square root and
# reciprocal square root issue at quarter rate: 4 lane-ops each)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


# Algorithmic VALU lane-operations per launch of every kernel kind.  Unit
# costs: an exponential of an FP64-reduced phase = 12 (FP64 product, round,
# subtract, convert = 4; sine + cosine at quarter rate = 8); a direction or
# Cartesian phase = 9 (2 FMA, 2 mul, 1 add, square root = 4); a real-by-
# complex multiply-add = 2; a complex product or multiply-add = 4.  Kernel
# values shared by a chunk of right-hand sides are counted once per chunk.
EXP, PHS, CRMAC, CMUL = 12, 9, 2, 4

# dense FP32 MFMA peak of MI355X
MFMA_FP32_PEAK_TFLOPS = 157.3


def mfma_init_flops(N: int, q: int) -> float:
    """FP32 flops of the initialisation's contraction for one right-hand
    side: per box B a real (q^2 x n_p) by complex (n_p x 64) product, i.e.
    2 x q^2 x n_p x 128 flops, and the n_p sum to N^2 over the boxes."""
    return 2.0 * q * q * 128 * N * N


def mfma_switch_flops(N: int, q: int) -> float:
    """FP32 flops of the matrix-core switch (either direction) for one
    right-hand side: per pair and direction node, a real q^2-by-q product
    with the real and imaginary parts of the weights, 2 x 2 q^3 flops; q
    nodes, N^2 pairs."""
    return 4.0 * q ** 4 * N * N


def switch_on_mfma(q: int, nrhs: int) -> bool:
    """The library runs the switch and its adjoint of complex64 batches of 32
    or more right-hand sides at q <= 9 on the matrix cores."""
    return q <= 9 and nrhs >= 32


def lane_ops(kind: str, N: int, q: int, s: int, nrhs: int, rc_switch: int = 8, rc_switch_adj: int = 4) -> float:
    n2 = float(N) * N
    h = q // 2
    m = 1 << s
    nA = 4 ** s
    if kind in ("plevel", "plevel_adj", "xlevel", "xlevel_adj"):
        shared = 5 * q * q * EXP + 3 * q * PHS if kind.startswith("p") else 5 * q * q * EXP + 2.5 * q * q * PHS
        per_rhs = 6 * q ** 3 * CRMAC + 5 * q * q * CMUL
        return n2 * (shared + nrhs * per_rhs)
    if kind in ("switch", "switch_adj"):
        rc = 1 if nrhs == 1 else (rc_switch if kind == "switch" else rc_switch_adj)
        chunks = -(-nrhs // rc)
        shared = q ** 3 * (PHS + (1 + h) * EXP)
        # forward: h paired updates (4 FMA) and one complex multiply-add per
        # (t, s2); adjoint: one conjugate product, h pairs of real-by-complex
        # multiply-adds and, for odd q, the middle row's addition
        per_rhs = q ** 3 * (4 * h + 4 + (2 * (q & 1) if kind == "switch_adj" else 0))
        return n2 * (chunks * shared + nrhs * per_rhs)
    if kind in ("init", "init_adj"):
        # per (A, source): phase + exponential + product + q^2 + q multiply-adds;
        # per (A, B box): q^2 remodulation exponentials and products
        per_rhs = nA * n2 * (PHS + EXP + CMUL + (q * q + q) * CRMAC) + nA * (n2 / nA) * q * q * (EXP + CMUL)
        return nrhs * per_rhs
    if kind in ("term", "term_adj"):
        # per (A, B): q^2 prefactors, the two 1-D passes, m^2 factors E(x, p0(B));
        # their kernel values (q^2 + m^2 phases and exponentials) once per
        # launch when several right-hand sides share them
        pairs = n2
        shared = (q * q + m * m) * (PHS + EXP)
        per_rhs = q * q * CMUL + (q * q * m + m * m * q) * CRMAC + m * m * CMUL
        return pairs * (shared * (1 if nrhs > 1 else nrhs) + nrhs * per_rhs)
    raise ValueError(kind)


def traffic_from_profiles(kernel: str, config: dict):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources and the same
    configuration (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if any(t.get("config", {}).get(k) != v for k, v in config.items()):
        return None
    h = hashlib.sha256()
    for f in sorted(t.get("sources", [])):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != t.get("sources_sha256"):
        return None
    return t.get("bytes_per_launch", {}).get(kernel)


def copy_calibration(nbytes: int = 1 << 30, reps: int = 5):
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    torch.cuda.set_device(0)
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}), flush=True)


def bench_3d(N: int, q: int, steps: int, warmup: int, rows: int):
    """The three-dimensional example (eq:ex3, Table 3 of the numerical
    section): forward applies of one white-noise input, FP32 weights, FP64
    phases; eq:err on ``rows`` sampled points against the direct sum."""
    import torch

    import paper_0809_0719_amd as fio
    from oracle import butterfly3 as B3
    torch.cuda.set_device(0)
    rng = np.random.default_rng(7)
    f_host = (rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))) / np.sqrt(2.0)
    plan = fio.Plan3(N, q, fio.SPHERES, dtype=torch.complex64)
    f = torch.as_tensor(f_host).to(torch.complex64).cuda()
    for _ in range(warmup):
        u = plan.apply(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        u = plan.apply(f)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # CPU baseline leg: the oracle's direct sum (numpy, FP64) at sampled points,
    # timed and extrapolated to all N^3 points; the same values give eq:err
    pts = np.sort(np.random.default_rng(107).choice(N ** 3, size=min(rows, N ** 3), replace=False))
    tc = time.perf_counter()
    ref = B3.direct3(N, B3.SPHERES, f.cpu().numpy().astype(np.complex128), pts)
    tcpu = time.perf_counter() - tc
    got = u.cpu().numpy().ravel()[pts]
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    cpu = {"value": len(pts) / (tcpu * N ** 3), "unit": "applies/s", "cores": 1, "kind": "oracle",
           "sample": f"FP64 direct sum (numpy, phases on one thread) at {len(pts)} of the {N ** 3} points, "
                     f"{tcpu:.2f} s; "
                     f"extrapolated x{N ** 3 / len(pts):.0f} to one full apply"}
    print(json.dumps({"metric": "3-D FIO applies/sec (eq:ex3)", "value": 1.0 / dt, "unit": "applies/s",
                      "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": dt * 1e3,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
                      "data": "synthetic", "rel_err_vs_direct_sum": err, "cpu_baseline": cpu,
                      "config": {"workload": f"eq:ex3 3-D N={N} q={q}", "N": N, "q": q}}), flush=True)


def bench_mixed(steps: int, warmup: int, nstreams: int):
    """The uneven batch: 32 problems drawn by the mixed-batch recipe (N in
    {128, 256, 512, 1024}, a tolerance in {1e-2, 1e-4, 1e-6} mapped to q =
    5 / 7 / 9, eta ~ U[0, 0.3]^2), one right-hand side each, through a Batch
    (internal streams) and, for comparison, one plan after another on one
    stream.  value = problems per second through the batch."""
    import torch

    import paper_0809_0719_amd as fio
    from workloads import mixed_batch, white_noise

    torch.cuda.set_device(0)
    qmap = {1e-2: 5, 1e-4: 7, 1e-6: 9}
    probs = mixed_batch(6, n=32)
    plans, fs = [], []
    for p in probs:
        plans.append(fio.Plan(p["N"], qmap[p["tol"]], fio.Phase(eta1=p["eta1"], eta2=p["eta2"])))
        fs.append(torch.as_tensor(white_noise(p["N"], p["f_seed"] % 100000)).to(torch.complex64).cuda())
    batch = fio.Batch(plans, nstreams=nstreams)
    outs = [torch.empty_like(f) for f in fs]

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t_batch = timed(lambda: batch.apply(fs, outs))
    t_serial = timed(lambda: [p.apply(f, out=o) for p, f, o in zip(plans, fs, outs)])
    counts = {}
    for p in probs:
        key = f"N{p['N']}-q{qmap[p['tol']]}"
        counts[key] = counts.get(key, 0) + 1
    print(json.dumps({"metric": "mixed-batch FIO applies/sec", "value": len(plans) / t_batch, "unit": "applies/s",
                      "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": t_batch * 1e3,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
                      "data": "synthetic", "serial_ms_per_step": t_serial * 1e3,
                      "speedup_vs_serial": t_serial / t_batch,
                      "config": {"workload": "32 problems, eq:ex1 with eta ~ U[0,0.3]^2", "nstreams": nstreams,
                                 "problems": counts}}), flush=True)


def bench_feature(kind: str, N: int, q: int, rank: int, steps: int, warmup: int):
    """One of the extensions at the benchmark's (N, q), timed beside the plain
    butterfly on the same plan:
    * dphase: u and its derivatives du/da1, du/da2 with respect to the ellipse
      scalings of one right-hand side (fio_apply_dphase, which takes the
      right-hand sides one at a time); value = such triples per second,
      against the plain single-right-hand-side forward;
    * amplitude: a separated amplitude a(x,k) = sum_t g_t(x) h_t(k) of the
      given rank, forward and adjoint (fio_apply_amplitude[_adjoint]); value
      = amplitude applies per second (a forward and an adjoint count two),
      against the rank right-hand sides of one batched forward and adjoint."""
    import torch

    import paper_0809_0719_amd as fio
    from workloads import amplitude_factors, white_noise

    torch.cuda.set_device(0)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    c64 = torch.complex64
    if kind == "dphase":
        plan = fio.Plan(N, q, fio.Phase(), dtype=c64)
        f = torch.as_tensor(white_noise(N, 3)).to(c64).cuda()
        u = torch.empty_like(f)
        t_feat = timed(lambda: plan.apply_dphase(f))
        t_plain = timed(lambda: plan.apply(f, out=u))
        value = 1 / t_feat
        metric, cfg = "FIO + phase-derivative applies/sec", {"nrhs": 1}
    else:
        plan = fio.Plan(N, q, fio.Phase(), dtype=c64, nrhs_max=rank)
        g_h, h_h = amplitude_factors(N, rank, 7)
        g, h = (torch.as_tensor(x).to(c64).cuda() for x in (g_h, h_h))
        f = torch.as_tensor(white_noise(N, 3)).to(c64).cuda()
        u = torch.empty_like(f)
        b = torch.empty_like(f)
        fr = torch.as_tensor(white_noise(N, 3, nrhs=rank)).to(c64).cuda()
        ur = torch.empty_like(fr)
        br = torch.empty_like(fr)

        def amp():
            plan.apply_amplitude(f, g, h, out=u)
            plan.adjoint_amplitude(u, g, h, out=b)

        def plain():
            plan.apply(fr, out=ur)
            plan.adjoint(ur, out=br)

        t_feat = timed(amp)
        t_plain = timed(plain)
        value = 2 / t_feat
        metric, cfg = "variable-amplitude FIO applies/sec", {"rank": rank}
    print(json.dumps({"metric": metric, "value": value, "unit": "applies/s", "n_gpus": 1, "steps": steps,
                      "warmup": warmup, "ms_per_step": t_feat * 1e3, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                      "plain_ms_per_step": t_plain * 1e3, "cost_vs_plain": t_feat / t_plain,
                      "config": dict({"workload": f"eq:ex1 FIO butterfly N={N} q={q}, {kind}"}, **cfg)}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--q", type=int, default=9)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--contract", choices=["fp", "bf16"], default="fp",
                    help="interpolation contractions: FP32 vector ALUs or BF16 MFMA (FP32 accumulation)")
    ap.add_argument("--rows", type=int, default=256, help="sampled points for eq:err (the paper's S)")
    ap.add_argument("--cpu-rows", type=int, default=3072,
                    help="sampled points of the CPU baseline (about 10 s of the FP64 direct sum)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dims", type=int, choices=[2, 3], default=2,
                    help="3: the three-dimensional example eq:ex3 (forward applies, --N3, --q3)")
    ap.add_argument("--mixed", action="store_true",
                    help="the uneven batch of 32 problems through a Batch, against one plan after another")
    ap.add_argument("--nstreams", type=int, default=4)
    ap.add_argument("--N3", type=int, default=64)
    ap.add_argument("--q3", type=int, default=7)
    ap.add_argument("--feature", choices=["dphase", "amplitude"],
                    help="time an extension at (--N, --q) beside the plain butterfly on the same plan")
    ap.add_argument("--rank", type=int, default=8, help="terms of the separated amplitude (--feature amplitude)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the butterfly pass here is a single-GPU build "
              "(--gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        copy_calibration()
        return
    if args.mixed:
        bench_mixed(args.steps, args.warmup, args.nstreams)
        return
    if args.dims == 3:
        bench_3d(args.N3, args.q3, args.steps, args.warmup, 64 if args.N3 <= 128 else 16)
        return
    if args.feature:
        bench_feature(args.feature, args.N, args.q, args.rank, args.steps, args.warmup)
        return

    import torch

    import paper_0809_0719_amd as fio
    from workloads import sample_points, white_noise

    torch.cuda.set_device(0)
    N, q, R = args.N, args.q, args.nrhs
    plan = fio.Plan(N, q, fio.Phase(), dtype=torch.complex64, nrhs_max=R, contract=args.contract)
    f_host = white_noise(N, 3, nrhs=R)
    f = torch.as_tensor(f_host).to(torch.complex64).cuda()
    u = torch.empty_like(f)
    g = torch.empty_like(f)
    torch.cuda.synchronize()

    def step():
        plan.apply(f, out=u)
        plan.adjoint(u, out=g)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_read()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile_read()
    plan.profile(False)
    total = t1 - t0
    ms_per_step = 1e3 * total / args.steps
    value = 2 * R * args.steps / total

    # plain single-RHS forward, for the comparison the metric names
    f1 = f[0]
    u1 = torch.empty_like(f1)
    for _ in range(2):
        plan.apply(f1, out=u1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    nplain = max(3, args.steps)
    for _ in range(nplain):
        plan.apply(f1, out=u1)
    torch.cuda.synchronize()
    plain = nplain / (time.perf_counter() - t2)

    # roofline of every kernel kind, and of the dominant one (largest share of
    # the timed region): algorithmic work per launch / average launch time.
    # VALU kernels: lane-operations against the VALU issue rate; the
    # initialisation on the matrix cores: its contraction's FP32 flops against
    # the FP32 MFMA peak.
    per_kind = {}
    for kind, (k_ms, k_n) in prof.items():
        if kind == "tables":
            continue
        avg_ms = k_ms / k_n
        if kind in ("init", "init_adj", "term", "term_adj"):
            per_launch_rhs = R * args.steps / k_n
        else:
            per_launch_rhs = R
        mfma_flops = None
        if kind in ("init", "init_adj") and per_launch_rhs > 1:
            mfma_flops = mfma_init_flops(N, q)
        elif kind in ("switch", "switch_adj") and switch_on_mfma(q, per_launch_rhs):
            mfma_flops = mfma_switch_flops(N, q)
        if mfma_flops is not None:
            ops = per_launch_rhs * mfma_flops
            ach = ops / (avg_ms * 1e-3) / 1e12
            per_kind[kind] = {"avg_ms": avg_ms, "launches": k_n, "bound": "mfma", "unit": "TFLOP/s",
                              "achieved": ach, "peak": MFMA_FP32_PEAK_TFLOPS, "frac": ach / MFMA_FP32_PEAK_TFLOPS}
        else:
            ops = lane_ops(kind, N, q, plan.s, per_launch_rhs)
            ach = ops / (avg_ms * 1e-3) / 1e12
            per_kind[kind] = {"avg_ms": avg_ms, "launches": k_n, "bound": "alu", "unit": "Tlane-op/s",
                              "achieved": ach, "peak": VALU_PEAK_TOPS, "frac": ach / VALU_PEAK_TOPS}
    kind = max(per_kind, key=lambda k: prof[k][0])
    kk = per_kind[kind]
    roof = {"bound": kk["bound"], "kernel": f"k_{kind}", "achieved": kk["achieved"], "peak": kk["peak"],
            "unit": kk["unit"], "frac": kk["frac"],
            "traffic": traffic_from_profiles(f"k_{kind}", {"N": N, "q": q, "nrhs": R, "dtype": "complex64",
                                                          "contract": args.contract}),
            "avg_ms": kk["avg_ms"], "launches": kk["launches"]}

    # accuracy: eq:err on sampled points against the FP64 direct sum, and the CPU baseline
    rows = sample_points(N, args.rows, seed=103)
    u0 = u[0].cpu().numpy().reshape(-1)[rows]
    rel_err = None
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import direct as D
        from oracle.build import build as build_oracle
        if not os.path.exists(os.path.join(ROOT, "oracle", "liborc_direct.so")):
            build_oracle()
        ud = D.forward(N, D.Phase(), f_host[0], rows)
        rel_err = D.rel_err(ud, u0.astype(np.complex128))
        crow = sample_points(N, args.cpu_rows, seed=104)
        tc = time.perf_counter()
        D.forward(N, D.Phase(), f_host[0], crow)
        tcpu = time.perf_counter() - tc
        t_full = tcpu * (N * N) / len(crow)
        cpu = {"value": 1.0 / t_full, "unit": "applies/s", "cores": D.num_threads(), "kind": "oracle",
               "sample": f"FP64 direct sum (eq:dfio) at {len(crow)} of the {N * N} points, all {N * N} "
                         f"sources, {tcpu:.2f} s; extrapolated x{N * N / len(crow):.0f} to one full apply"}

    out = {
        "metric": METRIC, "value": value, "unit": "applies/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"eq:ex1 FIO butterfly N={N} q={q} s={plan.s} lm={plan.lm}, "
                               f"complex white-noise f, forward+adjoint per step",
                   "N": N, "q": q, "nrhs": R, "s": plan.s, "lm": plan.lm, "phase_dtype": "f64",
                   "weight_dtype": "f32", "contract": args.contract},
        "plain_forward_applies_per_s": plain,
        "rel_err_vs_direct_sum": rel_err,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
        "kernel_roofline": per_kind,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
