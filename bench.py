"""Benchmark of the BSS-QMC sweep on one MI355X.

Workload: the 16 x 16 half-filled Hubbard model (t = 0.25, U = 2, beta = 20,
dtau = 0.5, Lambda = 40) with 128 independent Markov chains, delayed updates
of rank 32 and FP64 recomputation every 8 slices.  One step = one sweep of
every chain (128 x 256 x 40 = 1,310,720 Ising-field updates, both spins).

The headline path is mixed precision: FP32 G, flips, flushes and wraps in
the last fp32_slices slices of every block (chosen automatically from the
coupling, 2 at this U and dtau; an FP32 error made s wraps before a
recomputation grows ~e^{2 lambda} per wrap), FP64 elsewhere and for all
stabilisation.  The all-FP64 path is timed beside it, and so is the
all-FP32-bulk variant, whose drift shows why it is not the headline.

Prints one JSON line: updates/s of the headline path (inputs resident on the
GPU, chains equilibrated by the warm-up sweeps), the FP64 path and the
speedup; the relative wrap drift max|G_wrapped - G_fresh| / max(1, max|G|)
over the timed sweeps and max|dG| of sampled chains against the FP64 oracle;
the roofline of the dominant kernel family (HIP-event timings of the
library's own profiler on the stream it launches on) and the MFMA fraction of
the whole sweep; the oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HS field updates/sec at 16x16, β=20 (FP32+FP64-stab vs FP64), max|ΔG| vs oracle"
PEAK = {"f32": 157.3e12, "f64": 78.6e12}
HBM_PEAK = 8.0e12

# HBM bytes per launch (FETCH_SIZE x 1.9998 + WRITE_SIZE x 1.0, the scales a
# 256 MiB device copy gives) from the profiles/*hbm_traffic.md summaries of
# each hopping mode, valid while the kernel's source file is the one the
# counters were taken on (sha1 prefix); otherwise the traffic is reported as
# null.
_COMMON_TRAFFIC = {
    "flip_f64": (1.169e9, "k_flip.hip", "217c6bae88cd"),
    "flip_f32": (5.534e8, "k_flip.hip", "217c6bae88cd"),
    "qr_udv": (2.775e9, "k_qr.hip", "4ca8710ab0ca"),
    "qr_solve": (2.953e9, "k_qr.hip", "4ca8710ab0ca"),
}
# per launch of all 128 chains (the profile pass runs them as one shard)
TRAFFIC = {
    "dense": dict(_COMMON_TRAFFIC, **{
        "wrap_f32": (1.703e8, "k_gemm.hip", "57c2c9444073"),
        # mean over every full-size dispatch of the FP64 NN GEMM kernel (wraps,
        # block products and UDV products share it)
        "wrap_f64": (4.527e8, "k_gemm.hip", "57c2c9444073"),
    }),
    "kronecker": dict(_COMMON_TRAFFIC, **{
        # wraps: one right and one left Kronecker-factor product each (mean of the two)
        "wrap_f64": (2.725e8, "k_hop.hip", "990a600b01dc"),
        "wrap_f32": (1.358e8, "k_hop.hip", "990a600b01dc"),
        "hop_f64": (2.710e8, "k_hop.hip", "990a600b01dc"),
    }),
}


def traffic_of(fam: str, hopping: str):
    import hashlib
    if fam not in TRAFFIC[hopping]:
        return None
    val, src, sha = TRAFFIC[hopping][fam]
    path = os.path.join(ROOT, "paper_1504_05090_amd", "csrc", src)
    with open(path, "rb") as f:
        return val if hashlib.sha1(f.read()).hexdigest()[:12] == sha else None


def family_model(fam: str, N: int, mats: int, chains: int, acc: float, k: int, kron: bool = False):
    """Algorithmic work of one launch of a kernel family: (amount, peak per second, bound).

    MFMA-bound families count flops against the dense MFMA peak of their
    dtype; the Kronecker-factor products (the wraps with kron, block and
    measurement products) count the bytes they must move, X read and Y written
    once, against HBM bandwidth."""
    if fam == "hop_f64" or (kron and fam in ("wrap_f32", "wrap_f64")):
        esz = 4 if fam.endswith("f32") else 8
        return 2.0 * mats * N * N * esz, HBM_PEAK, "hbm"
    if fam in ("wrap_f32", "wrap_f64", "gemm_f64"):
        return 2.0 * N ** 3 * mats, PEAK[fam[-3:]], "mfma"     # one batched N x N x N product
    if fam == "qr_udv":
        return (8.0 / 3.0) * N ** 3 * mats, PEAK["f64"], "mfma"   # Householder R (4/3 N^3) + explicit Q (4/3 N^3)
    if fam == "qr_solve":
        return (13.0 / 3.0) * N ** 3 * mats, PEAK["f64"], "mfma"  # R (4/3), Q^T on N columns (2), back substitution (1)
    if fam in ("flip_f32", "flip_f64"):
        # per chain and slice, both spins: rank-k flushes 4 a N^3, row/column
        # corrections 4 a N^2 k (a = acceptance)
        return chains * (4.0 * acc * N ** 3 + 4.0 * acc * N ** 2 * k), PEAK[fam[-3:]], "mfma"
    return 0.0, None, None


def _family_roofline(fam, entry, N, mats, chains, acc, k, kron):
    launches, tot = entry
    amount, peak, bound = family_model(fam, N, mats, chains, acc, k, kron)
    if not amount or not launches:
        return {"launches": launches, "avg_launch_ms": tot / max(1, launches)}
    avg_ms = tot / launches
    return {"launches": launches, "avg_launch_ms": round(avg_ms, 5), "bound": bound,
            "frac": round(amount / (avg_ms / 1e3) / peak, 4)}


def run_path(bss, inst, precision, k, n_stab, steps, warmup, fp32_slices=0, profile=False, flags=0):
    import torch
    stream = torch.cuda.Stream()
    flags |= bss.FLAG_PROFILE if profile else 0
    ctx = bss.Context([inst], precision=precision, delay_k=k, n_stab=n_stab, flags=flags, stream=stream,
                      fp32_slices=fp32_slices)
    ctx.sweep(warmup)
    stream.synchronize()
    ctx.reset_stats()
    if profile:
        ctx.reset_profile()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.sweep(steps)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    st = ctx.stats()
    prof = ctx.profile() if profile else None
    return ctx, ms, st, prof


def run_batch(bss, insts, steps, warmup, flags):
    """Heterogeneous batch in one context: updates/s over all instances."""
    import torch
    stream = torch.cuda.Stream()
    ctx = bss.Context(insts, precision="fp64", stream=stream, flags=flags)
    ctx.sweep(warmup)
    ctx.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.sweep(steps)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    upd = sum(d["n_chains"] * d["L"] ** 2 * int(round(d["beta"] / d["dtau"])) for d in insts)
    graph = ctx.stats(0)["sweep_graph"]
    del ctx
    return upd * steps / (ms / 1e3), ms / steps, graph


def summary(st):
    return {"acceptance": st["accepted"] / max(1, st["proposals"]), "drift_rel_max": st["drift_rel_max"],
            "drift_rel_mean": st["drift_rel_mean"], "fp32_slices": st["fp32_slices"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--hopping", choices=["dense", "kronecker"], default="dense",
                    help="how the headline path applies e^{-+dtau K}: dense MFMA GEMMs (the benchmark's "
                         "definition) or the Kronecker-factor products")
    ap.add_argument("--no-kronecker", action="store_true",
                    help="skip the Kronecker-hopping line beside a dense headline")
    ap.add_argument("--cpu-chains", type=int, default=0, help="oracle chains for the CPU baseline (0 = cores)")
    ap.add_argument("--no-batch", action="store_true", help="skip the multigrid-batch measurement")
    ap.add_argument("--no-oracle-check", action="store_true", help="skip the sampled comparison with the oracle")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB between two device buffers three times (a plain copy kernel of "
                         "known size, to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the chains are independent Markov chains, which would be split "
              "by chain range over GPUs with no exchange during sweeps, but no multi-GPU path is built; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import paper_1504_05090_amd as bss
    from paper_1504_05090_amd.workloads import BASE_SEED, CONFIGS, T_HOP

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 x {args.calibrate_copy} MiB device-to-device", file=sys.stderr, flush=True)
        del src, dst

    cfg = CONFIGS["C4"]
    p = cfg["instances"][0]
    inst = dict(L=p["L"], U=p["U"], t=T_HOP, beta=p["beta"], dtau=p["dtau"], seed=BASE_SEED, n_chains=cfg["chains"])
    N, lam, C, k, n_stab = p["L"] ** 2, int(round(p["beta"] / p["dtau"])), cfg["chains"], cfg["k"], cfg["n_stab"]
    updates_per_step = C * N * lam
    print(f"[bench] 16x16 beta=20 dtau=0.5: {C} chains, k={k}, n_stab={n_stab}, {updates_per_step} updates/step, "
          f"{args.warmup} warm-up + {args.steps} timed sweeps", file=sys.stderr, flush=True)

    kron_head = args.hopping == "kronecker"
    hflags = bss.FLAG_KRONECKER_HOPPING if kron_head else 0
    ctx, ms, st, _ = run_path(bss, inst, "mixed", k, n_stab, args.steps, args.warmup, flags=hflags)
    value = updates_per_step * args.steps / (ms / 1e3)
    mixed = summary(st)
    m32 = mixed["fp32_slices"]
    print(f"[bench] mixed (FP32 in the last {m32} slices of each block): {ms / args.steps:.2f} ms/step, "
          f"{value:.4g} updates/s, {mixed}", file=sys.stderr, flush=True)

    # sampled chains against the oracle's G computed from scratch for the GPU's field
    max_dg = None
    try:
        if args.no_oracle_check:
            raise RuntimeError("not requested")
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

    fp64 = None
    fp64_value = None
    if not args.no_fp64:
        ctx64, ms64, st64, _ = run_path(bss, inst, "fp64", k, n_stab, args.steps, args.warmup, flags=hflags)
        fp64_value = updates_per_step * args.steps / (ms64 / 1e3)
        fp64 = dict(summary(st64), value=fp64_value, ms_per_step=ms64 / args.steps)
        print(f"[bench] fp64: {ms64 / args.steps:.2f} ms/step, {fp64_value:.4g} updates/s, {summary(st64)}",
              file=sys.stderr, flush=True)
        del ctx64
        # every slice in FP32: faster, but its drift is far outside any bound
        ctx32, ms32, st32, _ = run_path(bss, inst, "mixed", k, n_stab, max(2, args.steps // 2), 2,
                                        fp32_slices=n_stab, flags=hflags)
        all32 = dict(summary(st32), value=updates_per_step * max(2, args.steps // 2) / (ms32 / 1e3),
                     ms_per_step=ms32 / max(2, args.steps // 2))
        print(f"[bench] all slices FP32 (not valid at this coupling): {all32}", file=sys.stderr, flush=True)
        del ctx32
    else:
        all32 = None

    # the same sweeps with e^{-+dtau K} applied through its Kronecker factors
    # (an option of the library; the headline applies it as dense MFMA GEMMs)
    kron = None
    if not args.no_kronecker and not kron_head:
        ctxk, msk, stk, _ = run_path(bss, inst, "mixed", k, n_stab, args.steps, args.warmup,
                                     flags=bss.FLAG_KRONECKER_HOPPING)
        kval = updates_per_step * args.steps / (msk / 1e3)
        kron = dict(summary(stk), value=kval, ms_per_step=msk / args.steps, speedup_vs_headline=kval / value)
        del ctxk
        if not args.no_fp64:
            ctxk, msk, stk, _ = run_path(bss, inst, "fp64", k, n_stab, args.steps, args.warmup,
                                         flags=bss.FLAG_KRONECKER_HOPPING)
            kron["fp64_path"] = dict(summary(stk), value=updates_per_step * args.steps / (msk / 1e3),
                                     ms_per_step=msk / args.steps)
            del ctxk
        print(f"[bench] Kronecker hopping: {kron}", file=sys.stderr, flush=True)

    # per-kernel-family HIP-event timings of the headline path, with the
    # chains in one shard: with several shards their launches overlap, and an
    # event pair would time other shards' work as well
    psteps = max(2, args.steps // 2)
    saved = os.environ.get("BSS_SHARDS")
    os.environ["BSS_SHARDS"] = "1"
    try:
        ctxp, msp, stp, prof = run_path(bss, inst, "mixed", k, n_stab, psteps, 2, profile=True, flags=hflags)
    finally:
        if saved is None:
            del os.environ["BSS_SHARDS"]
        else:
            os.environ["BSS_SHARDS"] = saved
    del ctxp
    acc = stp["accepted"] / max(1, stp["proposals"])
    # the chains are split into shards with launches of their own: a launch
    # covers one shard's matrices
    shards = max(1, stp["shards"])
    Cl = C / shards
    mats = 2 * Cl
    fams = sorted(((f, v) for f, v in prof.items() if v[0] > 0), key=lambda kv: -kv[1][1])
    bound_time = 0.0
    for fam, (launches, tot) in fams:
        amount, pk, _ = family_model(fam, N, mats, Cl, acc, k, kron_head)
        if amount:
            bound_time += amount * launches / pk
    dom, (launches, tot) = fams[0]
    avg_ms = tot / max(1, launches)
    amount, peak, bound = family_model(dom, N, mats, Cl, acc, k, kron_head)
    achieved = amount / (avg_ms / 1e3) if amount else None
    scale = 1e9 if bound == "hbm" else 1e12
    roofline = {"kernel": dom, "bound": bound, "achieved": achieved / scale if achieved else None,
                "peak": peak / scale if peak else None, "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
                "frac": (achieved / peak) if (achieved and peak) else None, "traffic": traffic_of(dom, args.hopping),
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "avg_launch_ms": avg_ms, "launches": launches, "shards": shards,
                "matrices_per_launch": mats,
                "bound_time_fraction_of_sweep": bound_time / (msp / 1e3),
                "breakdown_ms_per_step": {kf: round(v[1] / psteps, 3) for kf, v in fams},
                "families": {kf: _family_roofline(kf, v, N, mats, Cl, acc, k, kron_head) for kf, v in fams}}
    print(f"[bench] profile ({msp / psteps:.2f} ms/step): {roofline['breakdown_ms_per_step']}", file=sys.stderr,
          flush=True)

    # the multigrid batch: 16 uneven instances x 32 chains, graph replays
    # against direct launches
    batch = None
    if not args.no_batch:
        c3 = CONFIGS["C3"]
        insts = [dict(L=q["L"], U=q["U"], t=T_HOP, beta=q["beta"], dtau=q["dtau"], seed=BASE_SEED,
                      n_chains=c3["chains"]) for q in c3["instances"]]
        v_graph, ms_graph, used_graph = run_batch(bss, insts, 5, 3, 0)
        v_direct, ms_direct, _ = run_batch(bss, insts, 5, 3, bss.FLAG_NO_GRAPH)
        batch = {"workload": "16 instances L in {6,8,10,12} x dtau in {0.4,0.5,0.625,0.8}, U=2, beta=20, "
                             "32 chains each, FP64, automatic k and n_stab",
                 "value": v_graph, "unit": "updates/s", "ms_per_step": ms_graph, "sweep_graph": used_graph,
                 "direct_launch_value": v_direct, "direct_launch_ms_per_step": ms_direct}
        print(f"[bench] batch C3: {batch}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores = min(len(os.sched_getaffinity(0)), 16)
        nch = args.cpu_chains or cores
        sec, used = oracle.run_chains(p["L"], p["U"], T_HOP, p["beta"], p["dtau"], BASE_SEED, nch, n_stab, 1, cores)
        cpu = {"value": nch * N * lam / sec, "unit": "updates/s", "cores": used, "kind": "oracle",
               "sample": f"{nch} chains x 1 sweep of the same 16x16 workload from the generator-drawn field "
                         f"(FP64 oracle: rank-1 updates, recomputation from scratch), {sec:.1f} s"}
        print(f"[bench] cpu oracle: {cpu}", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic (Markov chains from seeded Philox fields)",
        "config": {"workload": f"16x16 Hubbard BSS-QMC sweep, t=0.25, U=2, beta=20, dtau=0.5 (Lambda=40), "
                               f"{C} chains, k={k}, n_stab={n_stab}, FP32 in the last {m32} slices of each block, "
                               + ("e^{-+dtau K} through its Kronecker factors" if kron_head
                                  else "wraps and block products as dense MFMA GEMMs"),
                   "L": p["L"], "chains": C, "beta": p["beta"], "dtau": p["dtau"], "U": p["U"], "k": k,
                   "n_stab": n_stab, "fp32_slices": m32, "hopping": args.hopping, "shards": st["shards"]},
        "drift_rel_max": mixed["drift_rel_max"], "drift_rel_mean": mixed["drift_rel_mean"],
        "max_dG_vs_oracle_sweep_end": max_dg, "acceptance": mixed["acceptance"],
        "fp64_path": fp64, "speedup_vs_fp64": (value / fp64_value) if fp64_value else None,
        "all_fp32_bulk": all32, "kronecker_hopping": kron, "multigrid_batch": batch,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
