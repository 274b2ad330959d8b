"""Tuned launch parameters: a table written by bss_autotune, and its lookup.

The sweep's delay depth and block length change its cost, not its result
(up to rounding), and the best values depend on the device, the lattice, the
Trotter grid and the precision.  This module keeps one JSON table per device
architecture beside it (tuning_<arch>.json) with one entry per tuned
instance, keyed by (arch, N, Lambda, U, t, dtau, precision), and looks
entries up for new contexts:

    python -m paper_1504_05090_amd.tuning --workload C3

runs bss_autotune for every instance of a workload (paper_1504_05090_amd.workloads)
on the current device and merges the results into the table.  Each entry
also records what the tuner measured (ms per sweep of the trial chains, the
relative wrap drift, the number of candidates timed) and the bound it was
tuned under.  The tuner only tries block lengths whose slice product has a
condition estimate <= 1e12, the range in which the recomputed Green functions
are checked against the exact ones.
"""
from __future__ import annotations

import argparse
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
_KEYS = ("arch", "N", "Lambda", "U", "t", "dtau", "precision")


def table_path(arch: str) -> str:
    return os.path.join(_HERE, f"tuning_{arch}.json")


def device_arch() -> str:
    """gfx name of the current device (without feature suffixes)."""
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def load(arch: str) -> list:
    p = table_path(arch)
    if not os.path.exists(p):
        return []
    with open(p) as f:
        return json.load(f)["entries"]


def _key(arch, inst: dict, precision: str) -> tuple:
    lam = int(round(inst["beta"] / inst["dtau"]))
    return (arch, int(inst["L"]) ** 2, lam, round(float(inst["U"]), 12), round(float(inst.get("t", 0.25)), 12),
            round(float(inst["dtau"]), 12), precision)


def lookup(inst: dict, precision: str, arch: str | None = None, entries: list | None = None):
    """(delay_k, n_stab) tuned for this instance, or None."""
    arch = arch or device_arch()
    want = _key(arch, inst, precision)
    for e in (load(arch) if entries is None else entries):
        if tuple(e[k] for k in _KEYS) == want:
            return int(e["delay_k"]), int(e["n_stab"])
    return None


def apply(instances: list, precision: str, arch: str | None = None) -> list:
    """Copies of the instance dicts with the table's delay_k and n_stab set
    where the table has an entry (and a "tuned" flag on each)."""
    arch = arch or device_arch()
    entries = load(arch)
    out = []
    for d in instances:
        hit = lookup(d, precision, arch, entries)
        e = dict(d)
        e["tuned"] = hit is not None
        if hit is not None:
            e["delay_k"], e["n_stab"] = hit
        out.append(e)
    return out


def tune(instances: list, precision: str, drift_bound: float, warmup: int, trials: int) -> list:
    """Run bss_autotune for each instance; entries for the table."""
    import paper_1504_05090_amd as bss
    arch = device_arch()
    rows = []
    for d in instances:
        r = bss.autotune(d, precision=precision, drift_bound=drift_bound, warmup_sweeps=warmup, trial_sweeps=trials)
        k = _key(arch, d, precision)
        row = dict(zip(_KEYS, k))
        row.update(L=int(d["L"]), beta=float(d["beta"]), chains=int(d["n_chains"]), delay_k=r["delay_k"],
                   n_stab=r["n_stab"], fp32_slices=r["fp32_slices"], met_bound=r["met_bound"],
                   candidates=r["candidates"], ms_per_sweep=r["ms_per_sweep"], drift_rel_max=r["drift_rel_max"],
                   drift_bound=drift_bound, warmup_sweeps=warmup, trial_sweeps=trials)
        print(f"[tuning] {row}", flush=True)
        rows.append(row)
    return rows


def merge(arch: str, rows: list) -> str:
    """Replace or add the rows' keys in the table of arch; returns its path."""
    old = {tuple(e[k] for k in _KEYS): e for e in load(arch)}
    for r in rows:
        old[tuple(r[k] for k in _KEYS)] = r
    p = table_path(arch)
    with open(p, "w") as f:
        json.dump({"arch": arch, "written_by": "bss_autotune via paper_1504_05090_amd.tuning",
                   "entries": sorted(old.values(), key=lambda e: (e["N"], e["Lambda"], e["precision"]))}, f,
                  indent=1)
        f.write("\n")
    return p


def main():
    from paper_1504_05090_amd.workloads import BASE_SEED, CONFIGS, T_HOP
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", required=True, choices=sorted(CONFIGS))
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="default: the workload's own precision")
    ap.add_argument("--drift-bound", type=float, default=1e-5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--trials", type=int, default=3)
    a = ap.parse_args()
    w = CONFIGS[a.workload]
    prec = a.precision or w["precision"]
    insts = [dict(L=q["L"], U=q["U"], t=T_HOP, beta=q["beta"], dtau=q["dtau"], seed=BASE_SEED, n_chains=w["chains"])
             for q in w["instances"]]
    rows = tune(insts, prec, a.drift_bound, a.warmup, a.trials)
    print(f"[tuning] wrote {merge(device_arch(), rows)}", flush=True)


if __name__ == "__main__":
    main()
