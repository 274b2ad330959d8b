"""Write equilibrated Ising fields used as starting points by the GPU parity
tests.  Calls only the oracle: each field is the state of the oracle's chain
(key = (base seed + chain, 0)) after `sweeps` warm-up sweeps from its
generator-drawn start.

    python tests/golden/make_fields.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

BASE_SEED = 1504050900

FIELDS = {
    # file: (L, U, t, beta, dtau, n_stab, chain, sweeps)
    "field_L16_U2_b20_dt0.5_w20.npy": (16, 2.0, 0.25, 20.0, 0.5, 8, 0, 20),
    "field_L8_U2_b10_dt0.5_w50.npy": (8, 2.0, 0.25, 10.0, 0.5, 10, 0, 50),
}


def main():
    for name, (L, U, t, beta, dtau, n_stab, chain, sweeps) in FIELDS.items():
        c = oracle.Chain(L, U, t, beta, dtau, BASE_SEED, 0, chain, n_stab)
        c.sweep(sweeps)
        np.save(os.path.join(HERE, name), c.field())
        print(name, c.stats(), flush=True)


if __name__ == "__main__":
    main()
