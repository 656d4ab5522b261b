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

Printed on one JSON line: throughput; the roofline of every kernel and of
the dominant one -- algorithmic bytes and flops (the method's definition) per
launch over its time measured with HIP events recorded on the launch stream
inside the timed region, against the published HBM and FP32 peaks -- and the
end-to-end fraction; the relative error eq:err against the FP64 direct sum
for the first, middle and last right-hand side, forward on 256 sampled points
x and adjoint on 256 sampled frequencies k, with the verdict against the
metric's tolerance; and the CPU baseline: the direct-sum oracle timed on the
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
METRIC_TOL = 1e-4

# MI355X published peaks: HBM3E bandwidth and dense FP32 (matrix cores; the
# vector ALUs reach the same figure only with packed FP32, which the library
# does not use)
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0  # dense BF16 matrix-core peak (no sparsity)
CSIZE = 8  # bytes of one complex64 value


def algorithmic_work(kind: str, N: int, q: int, s: int, nrhs: int):
    """(HBM bytes, FP32 flops) one launch of `kind` needs by the method's
    definition, for `nrhs` right-hand sides in complex64.

    Bytes: every level, switch, initialisation and termination reads its
    input and writes its output once -- weights are N^2 q^2 complex values
    per right-hand side, sources and potentials N^2 (tables of a few KB and
    the initialisation's stored kernel values are not counted).

    Flops (real; a real-by-complex multiply-add is 4, a complex multiply-add
    8, a complex product 6), per pair and right-hand side:
      level (either half, either direction): the one-dimensional passes of
        the Kronecker sum, 6 q^3 real-by-complex multiply-adds, and 5 q^2
        complex products (prefactors and remodulation);
      switch: the q^2 x q^2 kernel of a pair (8 q^4 flops as a dense complex
        product), counted as the kernels execute it once the Chebyshev
        symmetry z_{q-1-j} = -z_j has halved it: 4 q^4 flops;
      initialisation: 4^s q^2 real-by-complex multiply-adds per source (the
        Lagrange weights against the kernel-weighted sources of every box A),
        q^2 complex products per pair;
      termination: q^2 2^s + q 4^s real-by-complex multiply-adds and
        q^2 + 4^s complex products per box pair."""
    n2 = float(N) * N
    W = n2 * q * q
    if kind in ("plevel", "plevel_adj", "xlevel", "xlevel_adj"):
        return 2 * W * CSIZE * nrhs, n2 * nrhs * (24 * q ** 3 + 30 * q * q)
    if kind in ("switch", "switch_adj"):
        return 2 * W * CSIZE * nrhs, n2 * nrhs * 4 * q ** 4
    if kind in ("init", "init_adj"):
        return (W + n2) * CSIZE * nrhs, n2 * nrhs * (4 * 4 ** s * q * q + 6 * q * q)
    if kind in ("term", "term_adj"):
        m = 1 << s
        return (W + n2) * CSIZE * nrhs, n2 * nrhs * (4 * (q * q * m + q * m * m) + 6 * (q * q + m * m))
    raise ValueError(kind)


def roofline_of(kind: str, avg_ms: float, launches: int, N: int, q: int, s: int, nrhs: int,
                contract: str = "fp") -> dict:
    """Both bounds of one kernel kind: achieved GB/s against the HBM peak and
    achieved TFLOP/s against the peak of the arithmetic it runs on (FP32, or
    BF16 matrix cores for the p-level under contract "bf16"); the binding one
    is the larger fraction (the bound the kernel is closest to)."""
    nbytes, flops = algorithmic_work(kind, N, q, s, nrhs)
    sec = avg_ms * 1e-3
    gbs, tfs = nbytes / sec / 1e9, flops / sec / 1e12
    peak = BF16_PEAK_TFLOPS if (contract == "bf16" and kind == "plevel") else FP32_PEAK_TFLOPS
    hf, ff = gbs / HBM_PEAK_GBS, tfs / peak
    out = {"avg_ms": avg_ms, "launches": launches, "nrhs": nrhs, "bytes": nbytes, "flops": flops,
           "hbm_gbs": gbs, "hbm_frac": hf, "fp32_tflops": tfs, "fp32_frac": ff,
           "bound_ms": max(nbytes / (HBM_PEAK_GBS * 1e9), flops / (peak * 1e12)) * 1e3}
    if peak != FP32_PEAK_TFLOPS:
        out.update(compute_peak_tflops=peak)
    if hf >= ff:
        out.update(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=hf)
    else:
        out.update(bound="mfma" if kind in mfma_kinds(q, s, nrhs, contract) else "alu", achieved=tfs, peak=peak,
                   unit="TFLOP/s", frac=ff)
    return out


def mfma_kinds(q: int, s: int, nrhs: int, contract: str = "fp") -> tuple:
    """Kernel kinds the library runs as FP32 matrix-core products for a
    complex64 plan: the initialisations at s = 3, q <= 9; the switches for
    chunks of 32 or more right-hand sides at q <= 9; with contract "mfma" also
    the p-levels and adjoint x-levels of such chunks; with contract "bf16" the
    p-levels (BF16 matrix cores, any number of right-hand sides)."""
    kinds = []
    if s == 3 and 3 <= q <= 9:
        kinds += ["init", "init_adj"]
    if 3 <= q <= 9 and nrhs >= 32:
        kinds += ["switch", "switch_adj"]
        if contract == "mfma":
            kinds += ["plevel", "xlevel_adj"]
    if contract == "bf16":
        kinds += ["plevel"]
    return tuple(kinds)


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


def bench_mixed(steps: int, warmup: int, nstreams: int, qmax: int = 16):
    """The uneven batch: 32 problems drawn by the mixed-batch recipe (N in
    {128, 256, 512, 1024}, a tolerance in {1e-2, 1e-4, 1e-6}, eta ~
    U[0, 0.3]^2), one right-hand side each.  q per (N, tolerance) class is
    the library's own choice (fio_select_q: the smallest q in [3, qmax] whose
    estimated eq:err on 64 sampled points is within the tolerance); a class
    no such q reaches is reported as unreached and runs at the q with the
    smallest estimate.  The batch runs through a Batch (internal streams)
    and, for comparison, one plan after another on one stream.  value =
    problems per second through the batch."""
    import torch

    import paper_0809_0719_amd as fio
    from workloads import mixed_batch, white_noise

    torch.cuda.set_device(0)
    probs = mixed_batch(6, n=32)
    classes = {}
    for p in probs:
        key = (p["N"], p["tol"])
        if key in classes:
            continue
        ph = fio.Phase(eta1=p["eta1"], eta2=p["eta2"])
        q, err, tried = fio.select_q(p["N"], ph, tol=p["tol"], qmin=3, qmax=qmax, nrows=64, seed=7)
        reached = err <= p["tol"]
        if not reached:
            q = min(tried, key=tried.get)
            err = tried[q]
        classes[key] = {"N": p["N"], "tol": p["tol"], "q": q, "est_err": err, "reached": bool(reached)}
        print(f"class N={p['N']} tol={p['tol']:g}: q={q} est_err={err:.3g} reached={reached}", flush=True)
    plans, fs = [], []
    for p in probs:
        q = classes[(p["N"], p["tol"])]["q"]
        plans.append(fio.Plan(p["N"], q, fio.Phase(eta1=p["eta1"], eta2=p["eta2"])))
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
        c = classes[(p["N"], p["tol"])]
        key = f"N{p['N']}-q{c['q']}"
        counts[key] = counts.get(key, 0) + 1
    unreached = [f"N{c['N']} tol {c['tol']:g} (best estimate {c['est_err']:.3g} at q={c['q']})"
                 for c in classes.values() if not c["reached"]]
    print(json.dumps({"metric": "mixed-batch FIO applies/sec", "value": len(plans) / t_batch, "unit": "applies/s",
                      "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": t_batch * 1e3,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
                      "data": "synthetic", "serial_ms_per_step": t_serial * 1e3,
                      "speedup_vs_serial": t_serial / t_batch,
                      "q_selection": "fio_select_q per (N, tolerance) class, q in [3, %d]" % qmax,
                      "classes": list(classes.values()), "unreached_classes": unreached,
                      "config": {"workload": "32 problems, eq:ex1 with eta ~ U[0,0.3]^2", "nstreams": nstreams,
                                 "problems": counts}}), flush=True)


def bench_feature(kind: str, N: int, q: int, rank: int, nrhs: int, steps: int, warmup: int):
    """One of the extensions at the benchmark's (N, q), timed beside the plain
    butterfly on the same plan:
    * dphase: u and its derivatives du/da1, du/da2 with respect to the ellipse
      scalings of `nrhs` right-hand sides at once (fio_apply_dphase on a plan
      of nrhs_max = nrhs, which takes them in even chunks of at most nrhs/3
      whose level kernels share their kernel values); value = such triples
      per second, against the plain batched forward of the same right-hand
      sides; the single-right-hand-side cost is reported beside it;
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
    extra = {}
    if kind == "dphase":
        plan = fio.Plan(N, q, fio.Phase(), dtype=c64, nrhs_max=nrhs)
        fr = torch.as_tensor(white_noise(N, 3, nrhs=nrhs)).to(c64).cuda()
        ur = torch.empty_like(fr)
        t_feat = timed(lambda: plan.apply_dphase(fr))
        t_plain = timed(lambda: plan.apply(fr, out=ur))
        t_one = timed(lambda: plan.apply_dphase(fr[0]))
        t_one_plain = timed(lambda: plan.apply(fr[0], out=ur[0]))
        value = nrhs / t_feat
        metric, cfg = "FIO + phase-derivative applies/sec", {"nrhs": nrhs}
        extra = {"single_rhs": {"ms": t_one * 1e3, "plain_ms": t_one_plain * 1e3,
                                "cost_vs_plain": t_one / t_one_plain}}
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
                      "plain_ms_per_step": t_plain * 1e3, "cost_vs_plain": t_feat / t_plain, **extra,
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
    ap.add_argument("--contract", choices=["fp", "mfma", "bf16"], default="fp",
                    help="level contractions: FP32 vector ALUs, FP32 matrix cores, or BF16 matrix cores "
                         "(FP32 accumulation)")
    ap.add_argument("--rows", type=int, default=256, help="sampled points for eq:err (the paper's S)")
    ap.add_argument("--cpu-rows", type=int, default=3072,
                    help="sampled points of the CPU baseline (about 10 s of the FP64 direct sum)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shape (no autotuning)")
    ap.add_argument("--dims", type=int, choices=[2, 3], default=2,
                    help="3: the three-dimensional example eq:ex3 (forward applies, --N3, --q3)")
    ap.add_argument("--mixed", action="store_true",
                    help="the uneven batch of 32 problems through a Batch, against one plan after another")
    ap.add_argument("--nstreams", type=int, default=4)
    ap.add_argument("--qmax", type=int, default=16, help="largest q --mixed may select")
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
        bench_mixed(args.steps, args.warmup, args.nstreams, args.qmax)
        return
    if args.dims == 3:
        bench_3d(args.N3, args.q3, args.steps, args.warmup, 64 if args.N3 <= 128 else 16)
        return
    if args.feature:
        bench_feature(args.feature, args.N, args.q, args.rank, args.nrhs, args.steps, args.warmup)
        return

    import torch

    import paper_0809_0719_amd as fio
    from workloads import sample_points, white_noise

    torch.cuda.set_device(0)
    N, q, R = args.N, args.q, args.nrhs
    plan = fio.Plan(N, q, fio.Phase(), dtype=torch.complex64, nrhs_max=R, contract=args.contract)
    # launch shape measured on this device before the timed region (the
    # shapes all give the same results)
    tune = plan.autotune(R) if not args.no_tune else {"candidates": 0, **plan.shape()}
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

    # roofline of every kernel kind and of the dominant one (largest share of
    # the timed region): algorithmic bytes and flops per launch (the method's
    # definition, see algorithmic_work) / the average launch time measured with
    # HIP events on the launch stream, against the published peaks
    per_kind = {}
    for kind, (k_ms, k_n) in prof.items():
        if kind == "tables":
            continue
        # levels and switches take the whole chunk per launch; the
        # initialisation and termination may take one right-hand side each
        nr = R * args.steps / k_n if kind in ("init", "init_adj", "term", "term_adj") else R
        per_kind[kind] = roofline_of(kind, k_ms / k_n, k_n, N, q, plan.s, nr, args.contract)
    kind = max(per_kind, key=lambda k: prof[k][0])
    kk = per_kind[kind]
    roof = {"bound": kk["bound"], "kernel": f"k_{kind}", "achieved": kk["achieved"], "peak": kk["peak"],
            "unit": kk["unit"], "frac": kk["frac"],
            "traffic": traffic_from_profiles(f"k_{kind}", {"N": N, "q": q, "nrhs": R, "dtype": "complex64",
                                                          "contract": args.contract}),
            "hbm_frac": kk["hbm_frac"], "fp32_frac": kk["fp32_frac"],
            "avg_ms": kk["avg_ms"], "launches": kk["launches"]}
    # end to end: the time the bounds allow for one step / the measured step
    bound_ms = sum(v["bound_ms"] * v["launches"] for v in per_kind.values()) / args.steps
    roof["end_to_end_frac"] = bound_ms / ms_per_step
    roof["end_to_end_bound_ms"] = bound_ms

    # accuracy: eq:err against the FP64 direct sum (the oracle's C loop) for
    # right-hand sides 0, 31 and 63 -- forward on 256 sampled x, adjoint on
    # 256 sampled k (the adjoint's input is the forward's output u) -- and the
    # CPU baseline
    errs = None
    cpu = None
    meets = None
    if not args.no_cpu_baseline:
        from oracle import direct as D
        from oracle.build import build as build_oracle
        if not os.path.exists(os.path.join(ROOT, "oracle", "liborc_direct.so")):
            build_oracle()
        rows = sample_points(N, args.rows, seed=103)
        cols = sample_points(N, args.rows, seed=105)
        errs = {"forward": {}, "adjoint": {}, "points": args.rows}
        for r in sorted({0, (R - 1) // 2, R - 1}):
            ud = D.forward(N, D.Phase(), f_host[r], rows)
            errs["forward"][str(r)] = D.rel_err(ud, u[r].cpu().numpy().reshape(-1)[rows].astype(np.complex128))
            ur = u[r].cpu().numpy().astype(np.complex128)
            gd = D.adjoint(N, D.Phase(), ur, cols)
            errs["adjoint"][str(r)] = D.rel_err(gd, g[r].cpu().numpy().reshape(-1)[cols].astype(np.complex128))
        worst = max(max(errs["forward"].values()), max(errs["adjoint"].values()))
        errs["max"] = worst
        meets = bool(worst <= METRIC_TOL)
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
        "launch_shape": tune,
        "plain_forward_applies_per_s": plain,
        "rel_err_vs_direct_sum": errs,
        "meets_metric_tolerance": meets,
        "metric_tolerance": METRIC_TOL,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
        "kernel_roofline": per_kind,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
