"""Benchmark of the BSS-QMC sweep on one MI355X.

Workload: the 16 x 16 half-filled Hubbard model (t = 0.25, U = 2, beta = 20,
dtau = 0.5, Lambda = 40) with 128 independent Markov chains, delayed updates
of rank 32 and FP64 recomputation every 8 slices.  One step = one sweep of
every chain (128 x 256 x 40 = 1,310,720 Ising-field updates, both spins).
The headline path is FP32 bulk (flips, rank-k flushes, wraps on FP32 MFMA)
with FP64 stabilisation; the all-FP64 path is timed beside it.

Prints one JSON line: updates/s of the headline path, the FP64 path and the
speedup, max|dG| of sampled chains against the FP64 oracle, the roofline of
the dominant kernel (HIP-event timings of the library's own profiler) and
the oracle timed on the host cores.
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

PEAK = {"fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12, "hbm": 8.0e12}


def algorithmic_flops(fam: str, N: int, mats: int) -> float:
    """FP64/FP32 flops one launch of a kernel family performs (per batch)."""
    if fam in ("wrap_gemm", "gemm_f64"):
        return 2.0 * N ** 3 * mats          # one batched N x N x N product
    if fam == "qr_udv":
        return (8.0 / 3.0) * N ** 3 * mats  # Householder R (4/3 N^3) + explicit Q (4/3 N^3)
    if fam == "qr_solve":
        return (13.0 / 3.0) * N ** 3 * mats  # R (4/3), Q^T on N columns (2), back substitution (1)
    return 0.0


def run_path(bss, inst, precision, k, n_stab, steps, warmup, profile=False):
    import torch
    stream = torch.cuda.Stream()
    flags = bss.FLAG_PROFILE if profile else 0
    ctx = bss.Context([inst], precision=precision, delay_k=k, n_stab=n_stab, flags=flags, stream=stream)
    ctx.sweep(warmup)
    stream.synchronize()
    if profile:
        ctx.reset_profile()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.sweep(steps)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    prof = ctx.profile() if profile else None
    return ctx, ms, prof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-chains", type=int, default=0, help="oracle chains for the CPU baseline (0 = cores)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: chains are independent and the build has no multi-GPU path "
              "(see the sharding note in DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1504_05090_amd as bss
    from paper_1504_05090_amd.workloads import BASE_SEED, CONFIGS, T_HOP

    cfg = CONFIGS["C4"]
    p = cfg["instances"][0]
    inst = dict(L=p["L"], U=p["U"], t=T_HOP, beta=p["beta"], dtau=p["dtau"], seed=BASE_SEED, n_chains=cfg["chains"])
    N, lam, C, k, n_stab = p["L"] ** 2, int(round(p["beta"] / p["dtau"])), cfg["chains"], cfg["k"], cfg["n_stab"]
    updates_per_step = C * N * lam
    print(f"[bench] 16x16 beta=20 dtau=0.5: {C} chains, k={k}, n_stab={n_stab}, {updates_per_step} updates/step",
          file=sys.stderr, flush=True)

    ctx, ms, _ = run_path(bss, inst, "mixed", k, n_stab, args.steps, args.warmup)
    value = updates_per_step * args.steps / (ms / 1e3)
    st = ctx.stats()
    acc = st["accepted"] / max(1, st["proposals"])
    print(f"[bench] mixed: {ms / args.steps:.2f} ms/step, {value:.4g} updates/s, acceptance {acc:.3f}, "
          f"drift max {st['drift_max']:.2e}", file=sys.stderr, flush=True)

    # sampled chains against the oracle's G computed from scratch for the GPU's field
    max_dg = None
    try:
        import oracle
        o = oracle.Chain(p["L"], p["U"], T_HOP, p["beta"], p["dtau"], BASE_SEED, 0, 0, n_stab)
        errs = []
        for c in (0, C - 1):
            f = ctx.field(0, c)
            for s in range(2):
                g = ctx.green(0, c, s)
                errs.append(float(np.max(np.abs(g - o.fresh_green(1, s, f)))))
        max_dg = max(errs)
    except Exception as e:  # noqa: BLE001
        print(f"[bench] oracle comparison skipped: {e}", file=sys.stderr)
    del ctx

    fp64_value = None
    if not args.no_fp64:
        ctx64, ms64, _ = run_path(bss, inst, "fp64", k, n_stab, max(2, args.steps // 2), 1)
        fp64_value = updates_per_step * max(2, args.steps // 2) / (ms64 / 1e3)
        print(f"[bench] fp64: {ms64 / max(2, args.steps // 2):.2f} ms/step, {fp64_value:.4g} updates/s",
              file=sys.stderr, flush=True)
        del ctx64

    # per-kernel HIP-event timings of the same workload
    ctxp, msp, prof = run_path(bss, inst, "mixed", k, n_stab, max(2, args.steps // 2), 1, profile=True)
    del ctxp
    fams = sorted(prof.items(), key=lambda kv: -kv[1][1])
    dom, (launches, tot) = fams[0]
    avg_ms = tot / max(1, launches)
    mats = 2 * C
    flops = algorithmic_flops(dom, N, mats)
    if dom == "wrap_gemm":
        bound, peak = "mfma", PEAK["fp32_mfma"]
    elif flops > 0:
        bound, peak = "mfma", PEAK["fp64_mfma"]
    else:
        bound, peak = "alu", None
    achieved = flops / (avg_ms / 1e3) if flops else None
    roofline = {"kernel": dom, "bound": bound, "achieved": achieved / 1e12 if achieved else None,
                "peak": peak / 1e12 if peak else None, "unit": "TFLOP/s",
                "frac": (achieved / peak) if (achieved and peak) else None, "traffic": None,
                "avg_launch_ms": avg_ms, "launches": launches,
                "breakdown_ms_per_step": {kf: round(v[1] / max(2, args.steps // 2), 3) for kf, v in fams}}
    print(f"[bench] profile: {roofline['breakdown_ms_per_step']}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0))
        cores = min(cores, 16)
        nch = args.cpu_chains or cores
        sec, used = oracle.run_chains(p["L"], p["U"], T_HOP, p["beta"], p["dtau"], BASE_SEED, nch, n_stab, 1, cores)
        cpu = {"value": nch * N * lam / sec, "unit": "updates/s", "cores": used, "kind": "oracle",
               "sample": f"{nch} chains x 1 sweep of the same 16x16 workload (FP64 oracle, rank-1 updates, "
                         f"full recomputation), {sec:.1f} s"}
        print(f"[bench] cpu oracle: {cpu}", file=sys.stderr, flush=True)

    out = {
        "metric": "HS field updates/sec at 16x16, beta=20 (FP32+FP64-stab vs FP64), max|dG| vs oracle",
        "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic (Markov chain from seeded Philox field)",
        "config": {"workload": "16x16 Hubbard BSS-QMC sweep, t=0.25, U=2, beta=20, dtau=0.5, 128 chains, "
                               "k=32, n_stab=8, mixed precision", "global_batch": C, "seq_len": lam,
                   "parallelism": "chains"},
        "fp64_value": fp64_value, "speedup_vs_fp64": (value / fp64_value) if fp64_value else None,
        "max_dG_vs_oracle": max_dg, "acceptance": acc,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
