"""Seeded synthetic workload draws.

Random draws only: this module holds none of the estimation method's
arithmetic, imports nothing else from the package and is shared by the tests
(which feed the oracle and the GPU path the same inputs) and the benchmark.
The recorded 10-degree EyeLink saccades of the paper's evaluation (Section 4)
are not available; these draws stand in for them:

* ``tiny``   one horizontal 10 deg saccade, T = 80 samples at 1 kHz, D = 43 ms.
* ``full``   2-D saccades, amplitude U[2, 30] deg, direction U[0, 360) deg,
             duration from the main sequence D = 2.2 ms/deg * A + 21 ms,
             T = ceil(D) samples.
* ``uneven`` as ``full`` but T ~ U{20..150} and D := T ms, and a per-saccade
             candidate count drawn from {4096, 16384, 65536}.

Each saccade gets 18 multipliers U[lo, hi] that scale the nominal OPC into the
"true" OPC used to synthesise its trace, and i.i.d. standard-normal noise
draws [T][C] that the caller scales by sigma.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 20070988
SIGMA = 0.05
UNEVEN_NCAND = (4096, 16384, 65536)


def draw_saccades(S: int, kind: str = "full", seed: int = BASE_SEED,
                  mult_range=(0.8, 1.2), sigma_range=None) -> dict:
    rng = np.random.default_rng([seed, S, {"tiny": 0, "full": 1, "uneven": 2}[kind]])
    if kind == "tiny":
        amp = np.full(S, 10.0)
        phi = np.zeros(S)
        dur = np.full(S, 43.0)
        T = np.full(S, 80, np.int32)
        C = 1
    else:
        amp = rng.uniform(2.0, 30.0, S)
        phi = rng.uniform(0.0, 360.0, S)
        if kind == "full":
            dur = 2.2 * amp + 21.0
            T = np.array([math.ceil(d) for d in dur], np.int32)
        elif kind == "uneven":
            T = rng.integers(20, 151, S).astype(np.int32)
            dur = T.astype(np.float64)
        else:
            raise ValueError(kind)
        C = 2
    seeds = rng.integers(0, 2**63 - 1, S, dtype=np.int64).astype(np.uint64)
    mult = rng.uniform(mult_range[0], mult_range[1], (S, 18))
    noise = [rng.standard_normal((int(t), C)) for t in T]
    sig = (np.full(S, SIGMA) if sigma_range is None
           else rng.uniform(sigma_range[0], sigma_range[1], S))
    ncand = (rng.choice(np.array(UNEVEN_NCAND), S) if kind == "uneven"
             else np.zeros(S, np.int64)).astype(np.int32)
    return dict(S=S, kind=kind, amp=amp, dir_deg=phi, dur_ms=dur, T=T, C=C, seed=seeds,
                mult=mult, noise=noise, sigma=sig, n_cand=ncand)


def subset(batch: dict, idx) -> dict:
    idx = list(idx)
    out = dict(batch)
    out["S"] = len(idx)
    for k in ("amp", "dir_deg", "dur_ms", "T", "seed", "mult", "sigma", "n_cand"):
        out[k] = batch[k][idx]
    out["noise"] = [batch["noise"][i] for i in idx]
    return out
