"""Benchmark of the BSS-QMC sweep on one MI355X.

Workload: the 16 x 16 half-filled Hubbard model (t = 0.25, U = 2, beta = 20,
dtau = 0.5, Lambda = 40) with 128 independent Markov chains, delayed updates
of rank 32 and FP64 recomputation every 8 slices.  One step = one sweep of
every chain (128 x 256 x 40 = 1,310,720 Ising-field updates, both spins).

The headline path is mixed precision with the automatic FP32 slice count:
FP32 G, flips, flushes and wraps in the last slices of every block, as many
as the library's drift controller allows (an FP32 error made s wraps before a
recomputation grows ~e^{2 lambda} per wrap; the controller starts in FP64 and
keeps the measured relative drift below 1e-3), FP64 everywhere else and for
all stabilisation.  The controller adapts the count during the warm-up sweeps
and then holds it, so the timed sweeps are replayed from one captured sweep
graph; the same path with the controller adapting after every timed sweep
(direct launches) and the all-FP64 path are timed beside it.

Prints one JSON line: updates/s of the headline path (everything resident on
the GPU, chains equilibrated by the warm-up sweeps) and of the FP64 path, the
relative wrap drift over the timed sweeps, the FP32 fraction, max|dG| of the
FP32 slices against the FP64 path on one identical history, the roofline of
the dominant kernel family in the timed configuration, the HBM rate of the
forced rank-1 path, the multigrid batch, and (the cpu_baseline leg) the oracle
timed on the host cores together with max|dG| of sampled sweep-end Green
functions against the oracle's.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HS field updates/sec at 16x16, β=20 (FP32+FP64-stab vs FP64), max|ΔG| vs oracle"
PEAK = {"f32": 157.3e12, "f64": 78.6e12}
HBM_PEAK = 8.0e12

# HBM bytes per launch in the timed configuration (one 128-chain shard, 256
# matrices), FETCH_SIZE x f + WRITE_SIZE x w with the scales f, w a device
# copy of known size gives (profiles/*_hbm_traffic.md), valid while the
# kernel's source file is the one the counters were taken on (sha1 prefix);
# otherwise null.
TRAFFIC = {
    "dense": {
        "qr_udv": (3.9631e9, "k_qr.hip", "758a4ba99fd6"),
        "lu_solve": (3.3188e9, "k_qr.hip", "758a4ba99fd6"),
        "flip_f64": (1.1113e9, "k_flip.hip", "dad164a0efd0"),
        "flip_f32": (4.870e8, "k_flip.hip", "dad164a0efd0"),
        # the FP64 NN GEMM kernel (wraps, block products and UDV products share it)
        "wrap_f64": (4.503e8, "k_gemm.hip", "57c2c9444073"),
        "gemm_f64": (4.503e8, "k_gemm.hip", "57c2c9444073"),
        "wrap_f32": (1.703e8, "k_gemm.hip", "57c2c9444073"),
    },
    "kronecker": {},
}


def traffic_of(fam: str, hopping: str):
    if fam not in TRAFFIC[hopping]:
        return None
    val, src, sha = TRAFFIC[hopping][fam]
    with open(os.path.join(ROOT, "paper_1504_05090_amd", "csrc", src), "rb") as f:
        return val if hashlib.sha1(f.read()).hexdigest()[:12] == sha else None


def family_model(fam: str, N: int, mats: float, chains: float, acc: float, k: int, kron: bool = False):
    """Algorithmic work of one launch of a kernel family: (amount, peak per second, bound).

    MFMA-bound families count flops against the dense MFMA peak of their
    dtype; the Kronecker-factor products count the bytes they must move, X
    read and Y written once, against HBM bandwidth."""
    if fam == "hop_f64" or (kron and fam in ("wrap_f32", "wrap_f64")):
        esz = 4 if fam.endswith("f32") else 8
        return 2.0 * mats * N * N * esz, HBM_PEAK, "hbm"
    if fam in ("wrap_f32", "wrap_f64", "gemm_f64"):
        return 2.0 * N ** 3 * mats, PEAK[fam[-3:]], "mfma"      # one batched N x N x N product
    if fam == "qr_udv":
        return (8.0 / 3.0) * N ** 3 * mats, PEAK["f64"], "mfma"  # Householder R (4/3 N^3) + explicit Q (4/3 N^3)
    if fam == "lu_solve":
        # LU (2/3 N^3), forward (N^3) and back (N^3) substitution on N right-hand sides
        return (8.0 / 3.0) * N ** 3 * mats, PEAK["f64"], "mfma"
    if fam in ("flip_f32", "flip_f64"):
        # per chain and slice, both spins: rank-k flushes 4 a N^3, row/column
        # corrections 4 a N^2 k (a = acceptance)
        return chains * (4.0 * acc * N ** 3 + 4.0 * acc * N ** 2 * k), PEAK[fam[-3:]], "mfma"
    return 0.0, None, None


def timed_sweeps(ctx, stream, n, measure=False):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.sweep(n, measure=measure)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def run_path(bss, inst, precision, k, n_stab, steps, warmup, fp32_slices=0, flags=0, drift_abort=None,
             adapt_sweeps=0):
    import torch
    stream = torch.cuda.Stream()
    ctx = bss.Context([inst], precision=precision, delay_k=k, n_stab=n_stab, flags=flags, stream=stream,
                      fp32_slices=fp32_slices, drift_abort=drift_abort, fp32_adapt_sweeps=adapt_sweeps)
    ctx.sweep(warmup)
    ctx.synchronize()
    ctx.reset_stats()
    ms = timed_sweeps(ctx, stream, steps)
    return ctx, stream, ms, ctx.stats()


def summary(st):
    return {"acceptance": st["accepted"] / max(1, st["proposals"]), "drift_rel_max": st["drift_rel_max"],
            "drift_rel_mean": st["drift_rel_mean"], "fp32_slices": st["fp32_slices"],
            "fp32_fraction": st["fp32_fraction"], "fp32_rejected": st["fp32_rejected"],
            "fp32_fused": st["fp32_fused"], "fp32_settled": st["fp32_settled"], "sweep_graph": st["sweep_graph"]}


def fp32_error_on_identical_history(bss, inst, field, k, n_stab, m32, n_slices):
    """max_ij |G_mixed - G_fp64| / max(1, max|G_fp64|) over the slices after
    which the mixed path holds G in FP32, on one history: the FP64 path
    records its accept decisions for n_slices slices from `field`, the mixed
    path (FP32 in the last m32 slices of each block) replays them."""
    one = dict(inst, n_chains=1)
    a = bss.Context([one], precision="fp64", delay_k=k, n_stab=n_stab, flags=bss.FLAG_RECORD_TRACE, trace_sweeps=1)
    a.set_field(field)
    ref = []
    for _ in range(n_slices):
        a.step_slices(1)
        ref.append([a.green(0, 0, s) for s in range(2)])
    tr = a.get_trace(1)
    b = bss.Context([one], precision="mixed", delay_k=k, n_stab=n_stab, flags=bss.FLAG_REPLAY_TRACE, trace_sweeps=1,
                    fp32_slices=m32)
    b.set_field(field)
    b.set_trace(tr, 1)
    lam = int(round(inst["beta"] / inst["dtau"]))

    def fp32_slice(l):
        return min(((l - 1) // n_stab + 1) * n_stab, lam) - l < m32

    worst, same = 0.0, True
    for l in range(1, n_slices + 1):
        b.step_slices(1)
        # G is held in FP32 after an FP32 slice that does not end a block, and
        # after a recomputation that precedes an FP32 slice
        ends_block = l % n_stab == 0 or l == lam
        in_fp32 = fp32_slice(l + 1) if ends_block else fp32_slice(l)
        for s in range(2):
            g, r = b.green(0, 0, s), ref[l - 1][s]
            if in_fp32:
                worst = max(worst, float(np.max(np.abs(g - r)) / max(1.0, np.max(np.abs(r)))))
            else:
                same = same and bool(np.array_equal(g, r))
    same = same and bool(np.array_equal(a.field(), b.field()))
    return worst, same


def profile_pass(bss, inst, k, n_stab, m32, ckpt, steps, flags):
    """Per-launch HIP-event timings of every kernel family in the timed
    configuration (same shards, the FP32 slice count the controller held),
    from the timed context's checkpoint: direct launches with an event pair
    around each launch on the stream it is issued on."""
    import torch
    stream = torch.cuda.Stream()
    prec = "mixed" if m32 > 0 else "fp64"
    ctx = bss.Context([inst], precision=prec, delay_k=k, n_stab=n_stab, flags=flags | bss.FLAG_PROFILE,
                      stream=stream, fp32_slices=m32)
    ctx.load(ckpt)
    ctx.sweep(1)
    ctx.synchronize()
    ctx.reset_stats()
    ctx.reset_profile()
    ms = timed_sweeps(ctx, stream, steps)
    st, prof = ctx.stats(), ctx.profile()
    del ctx
    return ms, st, prof


def rank1_pass(bss, inst, steps):
    """The forced rank-1 path (delay depth 1, FP64) on the same workload:
    every accepted flip reads and writes both spins' G (32 N^2 bytes), so its
    HBM rate is the measure of the flip kernel there."""
    import torch
    stream = torch.cuda.Stream()
    ctx = bss.Context([inst], precision="fp64", delay_k=1, n_stab=8, flags=bss.FLAG_PROFILE, stream=stream)
    ctx.sweep(2)
    ctx.synchronize()
    ctx.reset_stats()
    ctx.reset_profile()
    ms = timed_sweeps(ctx, stream, steps)
    st, prof = ctx.stats(), ctx.profile()
    del ctx
    N = inst["L"] ** 2
    acc = st["accepted"] / max(1, st["proposals"])
    launches, tot = prof["flip_f64"]
    chains_per_launch = inst["n_chains"] / st["shards"]
    bytes_per_launch = chains_per_launch * acc * N * 32.0 * N * N
    avg_s = tot / launches / 1e3
    return {"workload": "the headline workload with delay depth 1 (rank-1 Sherman-Morrison), FP64",
            "updates_per_s": inst["n_chains"] * N * int(round(inst["beta"] / inst["dtau"])) * steps / (ms / 1e3),
            "acceptance": acc, "flip_avg_launch_ms": tot / launches, "flip_launches": launches,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "achieved_GBps": bytes_per_launch / avg_s / 1e9, "peak_GBps": HBM_PEAK / 1e9,
            "frac": bytes_per_launch / avg_s / HBM_PEAK}


def run_batch(bss, insts, steps, warmup, flags):
    """Heterogeneous batch in one context: updates/s over all instances."""
    import torch
    stream = torch.cuda.Stream()
    ctx = bss.Context(insts, precision="fp64", stream=stream, flags=flags)
    ctx.sweep(warmup)
    ctx.synchronize()
    ms = timed_sweeps(ctx, stream, steps)
    upd = sum(d["n_chains"] * d["L"] ** 2 * int(round(d["beta"] / d["dtau"])) for d in insts)
    params = [dict(L=insts[j]["L"], dtau=insts[j]["dtau"], tuned=bool(insts[j].get("tuned", False)),
                   **{q: ctx.params(j)[q] for q in ("delay_k", "n_stab")}) for j in range(len(insts))]
    graph = ctx.stats(0)["sweep_graph"]
    del ctx
    return upd * steps / (ms / 1e3), ms / steps, graph, params


def post_processing(bss, ctx, p):
    """The library's analysis on the timed chains' own measurements (paper
    Sec. 3 and 4): G(tau_l, k) at k = (pi, 0) with its standard errors ->
    maximum-entropy spectrum at the historic alpha (eq. (4)) -> smooth G(tau)
    -> Matsubara transform (eq. (5)) -> Dyson self-energy (eq. (6), eps_k = 0,
    mu = 0: Re Sigma vanishes by particle-hole symmetry); C(r) -> xi.  Host
    code; each step timed.  Returns (summary, inputs for the oracle's turn)."""
    L, beta, dtau = p["L"], p["beta"], p["dtau"]
    lam = int(round(beta / dtau))
    gm, ge = ctx.gtau_k()
    kpi0 = L // 2                                    # k = (pi, 0): mx = L/2, my = 0
    tau = np.arange(lam + 1) * dtau
    G, sig = gm[:, kpi0].copy(), np.maximum(ge[:, kpi0], 1e-6)
    w = np.linspace(-4.0, 4.0, 161)
    m = np.full_like(w, 1.0 / 8.0)
    tau_f = np.linspace(0.0, beta, 401)
    out, t = {"k": "(pi, 0)", "tau_points": lam + 1, "omega_points": len(w), "matsubara_frequencies": 32}, {}
    inputs = dict(tau=tau, G=G, sig=sig, w=w, m=m, beta=beta, tau_f=tau_f, L=L)
    try:
        t0 = time.perf_counter()
        A, alpha, chi2 = bss.mem_spectrum(tau, G, sig, beta, w, m)
        t["mem_spectrum"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        Gs = bss.mem_green(beta, w, A, tau_f)
        t["mem_green"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        giw = bss.matsubara(tau_f, Gs, beta, 32)
        t["matsubara"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        sigma = bss.dyson(beta, 0.0, 0.0, giw)
        t["dyson"] = time.perf_counter() - t0
        out.update(alpha=alpha, chi2=chi2, spectral_weight=float(np.trapezoid(A, w)),
                   sum_rule_G0_plus_Gbeta=float(Gs[0] + Gs[-1]),
                   im_sigma_iw0=float(sigma[0].imag), max_abs_re_sigma=float(np.max(np.abs(sigma.real))),
                   max_abs_im_sigma=float(np.max(np.abs(sigma.imag))))
        inputs.update(A=A, alpha=alpha, Gs=Gs, giw=giw, sigma=sigma)
    except Exception as e:   # e.g. no historic alpha for these data
        out["mem_error"] = str(e)
    cm, _ = ctx.spin_corr()
    out.update(spin_corr_C0=float(cm[0]), spin_corr_C1=float(cm[1]))
    inputs["C"] = cm
    try:
        t0 = time.perf_counter()
        xi, _ = bss.correlation_length(L, cm)
        t["correlation_length"] = time.perf_counter() - t0
        out["xi"] = xi
    except Exception as e:   # no decay over the half lattice
        out["xi_error"] = str(e)
    out["library_ms"] = {k2: v * 1e3 for k2, v in t.items()}
    return out, inputs


def post_processing_oracle(post, inp):
    """The oracle's versions of the same steps on the same inputs, timed on the
    host, and their largest differences from the library's results."""
    from oracle import analysis as an
    from oracle import mem
    t = {}
    if "A" in inp:
        t0 = time.perf_counter()
        Ao, ao, _ = mem.spectrum(inp["tau"], inp["G"], inp["sig"], inp["beta"], inp["w"], inp["m"])
        t["mem_spectrum"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        Gso = mem.green(inp["tau_f"], inp["w"], Ao, inp["beta"])
        t["mem_green"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        giwo = an.matsubara(inp["tau_f"], Gso, inp["beta"], 32)
        t["matsubara"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        sigo = an.dyson(an.matsubara_frequencies(inp["beta"], 32), 0.0, 0.0, giwo)
        t["dyson"] = time.perf_counter() - t0
        big = Ao > 1e-6 * Ao.max()
        post["vs_oracle"] = {"alpha_rel": abs(inp["alpha"] - ao) / ao,
                             "A_rel_max": float(np.max(np.abs(inp["A"] - Ao)[big] / Ao[big])),
                             "G_smooth_abs_max": float(np.max(np.abs(inp["Gs"] - Gso))),
                             "sigma_abs_max": float(np.max(np.abs(inp["sigma"] - sigo)))}
    if "xi" in post:
        t0 = time.perf_counter()
        xio, _ = an.correlation_length(inp["C"], inp["L"])
        t["correlation_length"] = time.perf_counter() - t0
        post.setdefault("vs_oracle", {})["xi_rel"] = abs(post["xi"] - xio) / abs(xio)
    post["oracle_ms"] = {k2: v * 1e3 for k2, v in t.items()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline_leg(p, n_stab, ctx, C):
    """The oracle as it stands, on the host cores: updates/s on all cores of
    this process's share (one chain per core, 1 untimed + 1 timed sweep) and
    on one core (1 chain, 1 timed sweep).  Then the sampled parity check of
    the timed run's end state: sweep-end G of chains 0 and C-1 against the
    oracle's exact G (one slice per block) and its G at the same block length."""
    import oracle
    from paper_1504_05090_amd.workloads import BASE_SEED, T_HOP
    N, lam = p["L"] ** 2, int(round(p["beta"] / p["dtau"]))
    cores = min(len(os.sched_getaffinity(0)), 16)
    t0 = time.time()
    sec, used = oracle.run_chains(p["L"], p["U"], T_HOP, p["beta"], p["dtau"], BASE_SEED, cores, n_stab, 1,
                                  cores, n_warm=1)
    sec1, _ = oracle.run_chains(p["L"], p["U"], T_HOP, p["beta"], p["dtau"], BASE_SEED, 1, n_stab, 1, 1)
    wall = time.time() - t0
    cpu = {"value": cores * N * lam / sec, "unit": "updates/s", "cores": used, "kind": "oracle",
           "value_1_core": N * lam / sec1, "cpu_model": cpu_model(),
           "sample": f"{cores} chains x (1 untimed + 1 timed) sweep of the headline 16x16 workload, one chain "
                     f"per core, and 1 chain x 1 timed sweep on one core (FP64 oracle: rank-1 updates, full "
                     f"recomputation with column pivoting, gcc -O3, OpenMP over chains); {wall:.1f} s in all"}
    ex = oracle.Chain(p["L"], p["U"], T_HOP, p["beta"], p["dtau"], BASE_SEED, 0, 0, 1)
    same = oracle.Chain(p["L"], p["U"], T_HOP, p["beta"], p["dtau"], BASE_SEED, 0, 0, n_stab)
    d_ex, d_same = 0.0, 0.0
    for c in (0, C - 1):
        f = ctx.field(0, c)
        for s in range(2):
            g = ctx.green(0, c, s)
            for o, which in ((ex, "ex"), (same, "same")):
                r = o.fresh_green(1, s, f)
                d = float(np.max(np.abs(g - r)) / max(1.0, np.max(np.abs(r))))
                if which == "ex":
                    d_ex = max(d_ex, d)
                else:
                    d_same = max(d_same, d)
    return cpu, d_ex, d_same


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
    ap.add_argument("--all-fp32", action="store_true",
                    help="also time every slice in FP32 (not valid at this coupling: its drift is O(1))")
    ap.add_argument("--no-batch", action="store_true", help="skip the multigrid-batch measurement")
    ap.add_argument("--no-rank1", action="store_true", help="skip the forced rank-1 (k = 1) HBM measurement")
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
    from paper_1504_05090_amd import tuning
    from paper_1504_05090_amd.workloads import BASE_SEED, CONFIGS, T_HOP

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 x {args.calibrate_copy} MiB device-to-device", file=sys.stderr,
              flush=True)
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

    # 1. the headline: mixed precision, automatic FP32 slice count, adapted
    # during all but the last two warm-up sweeps and then held (the first held
    # sweep is captured, still inside the warm-up)
    settle = max(1, args.warmup - 2)
    ctx, stream, ms, st = run_path(bss, inst, "mixed", k, n_stab, args.steps, args.warmup, flags=hflags,
                                   adapt_sweeps=settle)
    value = updates_per_step * args.steps / (ms / 1e3)
    mixed = summary(st)
    m32 = mixed["fp32_slices"]
    print(f"[bench] mixed: {ms / args.steps:.2f} ms/step, {value:.4g} updates/s, {mixed}", file=sys.stderr,
          flush=True)
    # the same chains with measurement after every sweep (D and G(tau_l, k))
    n_meas = max(2, args.steps // 2)
    ms_meas = timed_sweeps(ctx, stream, n_meas, measure=True)
    value_meas = updates_per_step * n_meas / (ms_meas / 1e3)
    print(f"[bench] mixed with measurement: {ms_meas / n_meas:.2f} ms/step", file=sys.stderr, flush=True)
    post, post_in = post_processing(bss, ctx, p)
    print(f"[bench] post-processing of the measured G(tau, k) and C(r): {post}", file=sys.stderr, flush=True)
    ckpt = ctx.save()
    field0 = ctx.field(0, 0)

    # 2. FP32 error against the FP64 path on one identical history (two blocks)
    m32_err = max(1, m32) if m32 > 0 else 2
    fp32_err, fp64_slices_identical = fp32_error_on_identical_history(bss, inst, field0, k, n_stab, m32_err,
                                                                      2 * n_stab)
    print(f"[bench] FP32 slices ({m32_err} per block) vs FP64 path on one history: max rel|dG| {fp32_err:.3e}, "
          f"FP64 slices identical: {fp64_slices_identical}", file=sys.stderr, flush=True)

    # 3. the same path with the controller adapting after every sweep, timed
    # sweeps included (launched directly, one sweep at a time)
    ctxe, _, mse, ste = run_path(bss, inst, "mixed", k, n_stab, args.steps, args.warmup, flags=hflags)
    every = dict(summary(ste), value=updates_per_step * args.steps / (mse / 1e3), ms_per_step=mse / args.steps)
    del ctxe
    print(f"[bench] mixed, controller adapting after every sweep: {mse / args.steps:.2f} ms/step", file=sys.stderr,
          flush=True)

    # 4. the FP64 path
    fp64, fp64_value = None, None
    if not args.no_fp64:
        ctx64, _, ms64, st64 = run_path(bss, inst, "fp64", k, n_stab, args.steps, args.warmup, flags=hflags)
        fp64_value = updates_per_step * args.steps / (ms64 / 1e3)
        fp64 = dict(summary(st64), value=fp64_value, ms_per_step=ms64 / args.steps)
        print(f"[bench] fp64: {ms64 / args.steps:.2f} ms/step, {fp64_value:.4g} updates/s", file=sys.stderr,
              flush=True)
        del ctx64
    all32 = None
    if args.all_fp32:
        ctx32, _, ms32, st32 = run_path(bss, inst, "mixed", k, n_stab, max(2, args.steps // 2), 2,
                                        fp32_slices=n_stab, flags=hflags, drift_abort=0.0)
        all32 = dict(summary(st32), value=updates_per_step * max(2, args.steps // 2) / (ms32 / 1e3),
                     ms_per_step=ms32 / max(2, args.steps // 2), valid=False)
        print(f"[bench] all slices FP32 (not valid at this coupling): {all32}", file=sys.stderr, flush=True)
        del ctx32

    # 5. the Kronecker-factor option of e^{-+dtau K} on the same workload
    kron = None
    if not args.no_kronecker and not kron_head:
        ctxk, _, msk, stk = run_path(bss, inst, "mixed", k, n_stab, args.steps, args.warmup,
                                     flags=bss.FLAG_KRONECKER_HOPPING, adapt_sweeps=settle)
        kval = updates_per_step * args.steps / (msk / 1e3)
        kron = dict(summary(stk), value=kval, ms_per_step=msk / args.steps, speedup_vs_headline=kval / value)
        del ctxk
        print(f"[bench] Kronecker hopping: {kron}", file=sys.stderr, flush=True)

    # 6. roofline of the dominant kernel family in the timed configuration
    psteps = max(2, args.steps // 2)
    msp, stp, prof = profile_pass(bss, inst, k, n_stab, m32, ckpt, psteps, hflags)
    acc = stp["accepted"] / max(1, stp["proposals"])
    shards = max(1, stp["shards"])
    Cl = C / shards
    mats = 2 * Cl
    fams = sorted(((f, v) for f, v in prof.items() if v[0] > 0), key=lambda kv: -kv[1][1])
    bound_time = 0.0
    families = {}
    for fam, (launches, tot) in fams:
        amount, pk, bound = family_model(fam, N, mats, Cl, acc, k, kron_head)
        entry = {"launches": launches, "ms_per_step": round(tot / psteps, 3),
                 "avg_launch_ms": round(tot / launches, 5)}
        if amount:
            bound_time += amount * launches / pk
            entry.update(bound=bound, frac=round(amount / (tot / launches / 1e3) / pk, 4))
        families[fam] = entry
    dom, (launches, tot) = fams[0]
    avg_ms = tot / launches
    amount, peak, bound = family_model(dom, N, mats, Cl, acc, k, kron_head)
    achieved = amount / (avg_ms / 1e3) if amount else None
    scale = 1e9 if bound == "hbm" else 1e12
    roofline = {"kernel": dom, "bound": bound, "achieved": achieved / scale if achieved else None,
                "peak": peak / scale if peak else None, "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
                "frac": (achieved / peak) if (achieved and peak) else None,
                # the counters were taken on 256-matrix launches
                "traffic": traffic_of(dom, args.hopping) if mats == 256 else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "algorithmic_per_launch": amount, "avg_launch_ms": avg_ms, "launches": launches,
                "shards": shards, "matrices_per_launch": mats, "fp32_slices": m32,
                "profile_pass_ms_per_step": msp / psteps,
                "bound_time_fraction_of_sweep": bound_time / (msp / 1e3), "families": families}
    print(f"[bench] profile pass ({msp / psteps:.2f} ms/step): dominant {dom}, {families}", file=sys.stderr,
          flush=True)

    # 7. the forced rank-1 path: HBM rate of the flip kernel
    rank1 = None if args.no_rank1 else rank1_pass(bss, inst, 2)
    if rank1:
        print(f"[bench] rank-1 path: {rank1}", file=sys.stderr, flush=True)

    # 8. the multigrid batch: 16 uneven instances x 32 chains
    batch = None
    if not args.no_batch:
        c3 = CONFIGS["C3"]
        insts = [dict(L=q["L"], U=q["U"], t=T_HOP, beta=q["beta"], dtau=q["dtau"], seed=BASE_SEED,
                      n_chains=c3["chains"]) for q in c3["instances"]]
        # per-instance delay depth and block length from the table bss_autotune
        # wrote for this device (paper_1504_05090_amd/tuning_<arch>.json)
        tinsts = tuning.apply(insts, "fp64")
        v_graph, ms_graph, used_graph, params = run_batch(bss, tinsts, 5, 3, 0)
        v_direct, ms_direct, _, _ = run_batch(bss, tinsts, 5, 3, bss.FLAG_NO_GRAPH)
        v_auto, ms_auto, _, _ = run_batch(bss, insts, 5, 3, 0)
        batch = {"workload": "16 instances L in {6,8,10,12} x dtau in {0.4,0.5,0.625,0.8}, U=2, beta=20, "
                             "32 chains each, FP64", "value": v_graph, "unit": "updates/s",
                 "ms_per_step": ms_graph, "sweep_graph": used_graph,
                 "parameters": f"tuned: {sum(p['tuned'] for p in params)} of {len(params)} instances from "
                               f"tuning_{tuning.device_arch()}.json (bss_autotune), the rest automatic",
                 "direct_launch_value": v_direct, "direct_launch_ms_per_step": ms_direct,
                 "automatic_parameters_ms_per_step": ms_auto, "automatic_parameters_value": v_auto,
                 "instances": params}
        print(f"[bench] batch: {batch}", file=sys.stderr, flush=True)

    # 9. the cpu_baseline leg: the oracle on the host, and the sampled check
    cpu, d_exact, d_same = None, None, None
    if not args.no_cpu_baseline:
        cpu, d_exact, d_same = cpu_baseline_leg(p, n_stab, ctx, C)
        post_processing_oracle(post, post_in)
        print(f"[bench] cpu oracle: {cpu}; sampled sweep-end max rel|dG|: vs exact {d_exact:.3e}, vs oracle at "
              f"n_stab={n_stab} {d_same:.3e}", file=sys.stderr, flush=True)
    del ctx

    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic (Markov chains from seeded Philox fields)",
        "config": {"workload": f"16x16 Hubbard BSS-QMC sweep, t=0.25, U=2, beta=20, dtau=0.5 (Lambda=40), "
                               f"{C} chains, k={k}, n_stab={n_stab}, FP32 in the last slices of each block as the "
                               f"drift controller allows (target 1e-3; adapted during the first {settle} warm-up "
                               f"sweeps, then held: captured sweep graph), "
                               + ("e^{-+dtau K} through its Kronecker factors" if kron_head
                                  else "wraps and block products as dense MFMA GEMMs"),
                   "L": p["L"], "chains": C, "beta": p["beta"], "dtau": p["dtau"], "U": p["U"], "k": k,
                   "n_stab": n_stab, "fp32_slices_final": m32, "hopping": args.hopping, "shards": st["shards"],
                   "fp32_adapt_sweeps": settle, "sweep_graph": st["sweep_graph"]},
        "drift_rel_max": mixed["drift_rel_max"], "drift_rel_mean": mixed["drift_rel_mean"],
        "fp32_drift_bound": 1e-3, "fp32_fraction": mixed["fp32_fraction"], "acceptance": mixed["acceptance"],
        "fp32_rejected_ratios": mixed["fp32_rejected"], "fp32_fused": mixed["fp32_fused"],
        "fp32_max_dG_vs_fp64_path": fp32_err, "fp32_slices_for_that_check": m32_err,
        "fp64_slices_bit_identical": fp64_slices_identical,
        "max_dG_vs_oracle_sweep_end": d_exact, "max_dG_vs_oracle_same_n_stab": d_same,
        "value_with_measurement": value_meas, "ms_per_step_with_measurement": ms_meas / n_meas,
        "controller_every_sweep": every, "fp64_path": fp64,
        "speedup_vs_fp64": (value / fp64_value) if fp64_value else None,
        "all_fp32_bulk": all32, "kronecker_hopping": kron, "rank1_path": rank1, "multigrid_batch": batch,
        "roofline": roofline, "cpu_baseline": cpu, "post_processing": post,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
