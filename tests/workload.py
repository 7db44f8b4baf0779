"""Test inputs: synth draws -> FP32 traces built by the oracle (never by the GPU path)."""
import numpy as np

import oracle
from paper_2007_09884_amd import synth


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def make_batch(S, kind="full", seed=synth.BASE_SEED, sigma=None):
    """Returns (batch dict with float32-rounded amp/dir/dur, list of [T][C] float32 traces)."""
    b = synth.draw_saccades(S, kind, seed=seed)
    b["amp"], b["dir_deg"], b["dur_ms"] = f32(b["amp"]), f32(b["dir_deg"]), f32(b["dur_ms"])
    traces = []
    for i in range(S):
        T = int(b["T"][i])
        p = oracle.true_opc(b["mult"][i], b["dur_ms"][i])
        sg = b["sigma"][i] if sigma is None else sigma
        traces.append(oracle.make_target(p, b["amp"][i], b["dir_deg"][i], T, b["C"], b["noise"][i], sg))
    return b, traces


def records(b, opmm, n_cand=None):
    S = b["S"]
    return opmm.saccade_records(b["T"], b["C"], b["amp"], b["dir_deg"], b["dur_ms"], b["seed"],
                                n_cand=n_cand)
