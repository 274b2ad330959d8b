"""Run one of the configured workloads and report per instance.

    python -m paper_1504_05090_amd.run --workload C5 [--warmup W] [--sweeps S]

creates the workload's batch (paper_1504_05090_amd.workloads), sweeps it W
times unmeasured (in mixed precision the drift controller adapts its FP32
count during these sweeps and then holds it), resets the statistics, then
times S sweeps with measurement after each, and prints one JSON line per
instance: the resolved delay depth, block length and FP32 count, the
acceptance, the relative wrap drift (max and mean over the measured
sweeps), the double occupancy and the largest standard error of G(tau_l, k)
over tau_l and k (errors over chains), followed by a JSON line for the whole
batch (ms per measured sweep, updates/s).
"""
from __future__ import annotations

import argparse
import json

import numpy as np


def run(name: str, warmup: int | None = None, sweeps: int | None = None, chains: int | None = None) -> list:
    import torch

    import paper_1504_05090_amd as bss
    from paper_1504_05090_amd.workloads import BASE_SEED, CONFIGS, T_HOP

    w = CONFIGS[name]
    warmup = w["warmup"] if warmup is None else warmup
    sweeps = w["sweeps"] if sweeps is None else sweeps
    chains = w["chains"] if chains is None else chains
    insts = [dict(L=q["L"], U=q["U"], t=T_HOP, beta=q["beta"], dtau=q["dtau"], seed=BASE_SEED, n_chains=chains)
             for q in w["instances"]]
    stream = torch.cuda.Stream()
    ctx = bss.Context(insts, precision=w["precision"], delay_k=w["k"], n_stab=w["n_stab"], stream=stream,
                      fp32_adapt_sweeps=max(1, warmup - 1) if w["precision"] == "mixed" else 0)
    ctx.sweep(warmup)
    ctx.synchronize()
    ctx.reset_stats()
    ctx.reset_measurements()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.sweep(sweeps, measure=True)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / max(1, sweeps)
    rows = []
    updates = 0
    for j, d in enumerate(insts):
        p, st = ctx.params(j), ctx.stats(j)
        dm, de = ctx.double_occ(j)
        _, gerr = ctx.gtau_k(j)
        updates += chains * p["N"] * p["Lambda"]
        rows.append(dict(L=d["L"], U=d["U"], beta=d["beta"], dtau=d["dtau"], chains=chains, N=p["N"],
                         Lambda=p["Lambda"], delay_k=st["delay_k"], n_stab=st["n_stab"],
                         fp32_slices=st["fp32_slices"], fp32_settled=st["fp32_settled"],
                         fp32_fused=st["fp32_fused"], acceptance=st["accepted"] / max(1, st["proposals"]),
                         drift_rel_max=st["drift_rel_max"], drift_rel_mean=st["drift_rel_mean"],
                         double_occ=dm, double_occ_err=de, gtau_k_err_max=float(np.max(gerr))))
    rows.append(dict(workload=name, warmup=warmup, measured_sweeps=sweeps, ms_per_sweep=ms,
                     updates_per_s=updates / (ms / 1e3), sweep_graph=ctx.stats(0)["sweep_graph"]))
    return rows


def main():
    from paper_1504_05090_amd.workloads import CONFIGS
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", required=True, choices=sorted(CONFIGS))
    ap.add_argument("--warmup", type=int, default=None, help="default: the workload's own")
    ap.add_argument("--sweeps", type=int, default=None, help="measured sweeps; default: the workload's own")
    ap.add_argument("--chains", type=int, default=None, help="chains per instance; default: the workload's own")
    a = ap.parse_args()
    for r in run(a.workload, a.warmup, a.sweeps, a.chains):
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
