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
host on those 256 points and extrapolated to all N^2 points.
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


def switch_lane_ops_per_pair(q: int) -> int:
    """Minimum VALU lane-ops of one switch pair (eq:alg2m) as the kernel
    formulates it: per (t, s2) one direction phase G = Phi(x_t, e(theta_s2))
    (2 FMA, 2 mul, 1 add, 1 square root = 9), 1 + q//2 exponentials (FP64
    product, round, subtract, convert = 4; sine + cosine = 8), q//2 paired
    complex-by-(real,imag) updates (4 FMA) and one complex multiply-add (4)."""
    h = q // 2
    return q ** 3 * (9 + 12 * (1 + h) + 4 * h + 4)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--q", type=int, default=9)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--contract", choices=["fp", "bf16"], default="fp",
                    help="interpolation contractions: FP32 vector ALUs or BF16 MFMA (FP32 accumulation)")
    ap.add_argument("--rows", type=int, default=256, help="sampled points for eq:err and the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the butterfly pass here is a single-GPU build "
              "(--gpus 1).", file=sys.stderr)
        sys.exit(2)

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

    # roofline of the dominant kernel (largest share of the timed region)
    kind = max(prof, key=lambda k: prof[k][0])
    k_ms, k_n = prof[kind]
    avg_ms = k_ms / k_n
    if kind in ("switch", "switch_adj"):
        ops = switch_lane_ops_per_pair(q) * N * N
        achieved = ops / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": f"k_{kind}", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                "avg_ms": avg_ms, "launches": k_n}
    else:
        roof = {"bound": "alu", "kernel": f"k_{kind}", "achieved": None, "peak": VALU_PEAK_TOPS,
                "unit": "Tlane-op/s", "frac": None, "traffic": None, "avg_ms": avg_ms, "launches": k_n}

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
        tc = time.perf_counter()
        ud = D.forward(N, D.Phase(), f_host[0], rows)
        tcpu = time.perf_counter() - tc
        rel_err = D.rel_err(ud, u0.astype(np.complex128))
        t_full = tcpu * (N * N) / len(rows)
        cpu = {"value": 1.0 / t_full, "unit": "applies/s", "cores": D.num_threads(), "kind": "oracle",
               "sample": f"FP64 direct sum (eq:dfio) at {len(rows)} of the {N * N} points, all {N * N} "
                         f"sources, {tcpu:.2f} s; extrapolated x{N * N // len(rows)} to one full apply"}

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
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
