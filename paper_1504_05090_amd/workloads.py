"""Seeded synthetic workloads shared by the tests, the benchmark and the
smoke check.  This module holds parameters and seeded random inputs only --
none of the method's arithmetic.

The Markov chain itself is the workload (there is no dataset): the half-filled
Hubbard model with t = 0.25 on periodic L x L clusters (Sec. 2 of the paper),
the Ising field drawn uniformly +-1 from the counter-based generator keyed by
(base seed + chain, instance).
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 1504050900
T_HOP = 0.25

# name -> instance list + run parameters.  precision: "fp64" or "mixed"
# (FP32 bulk with FP64 stabilisation).
CONFIGS = {
    "C1": dict(instances=[dict(L=4, U=2.0, beta=4.0, dtau=0.5)], chains=1,
               precision="fp64", k=1, n_stab=4, warmup=200, sweeps=1000),
    "C2": dict(instances=[dict(L=8, U=2.0, beta=10.0, dtau=0.5)], chains=64,
               precision="fp64", k=16, n_stab=10, warmup=50, sweeps=500),
    "C3": dict(instances=[dict(L=L, U=2.0, beta=20.0, dtau=dt)
                          for L in (6, 8, 10, 12) for dt in (0.4, 0.5, 0.625, 0.8)],
               chains=32, precision="fp64", k=0, n_stab=0, warmup=20, sweeps=100),
    "C4": dict(instances=[dict(L=16, U=2.0, beta=20.0, dtau=0.5)], chains=128,
               precision="mixed", k=32, n_stab=8, warmup=20, sweeps=50),
    "C5": dict(instances=[dict(L=L, U=U, beta=40.0, dtau=dt)
                          for L in (16, 20) for U in (1.0, 2.0) for dt in (0.4, 0.5)],
               chains=64, precision="mixed", k=32, n_stab=0, warmup=10, sweeps=20),
}


def n_slices(beta: float, dtau: float) -> int:
    return int(round(beta / dtau))


def random_field(L: int, beta: float, dtau: float, seed: int) -> np.ndarray:
    """A uniform +-1 Ising field [Lambda, N] (int8) from numpy's generator,
    for tests that set a field explicitly."""
    rng = np.random.default_rng(seed)
    lam = n_slices(beta, dtau)
    return (2 * rng.integers(0, 2, size=(lam, L * L)) - 1).astype(np.int8)
