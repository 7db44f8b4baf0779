"""The C-ABI library loads on a CPU-only host and exports every symbol the header declares.
No compute calls here (they need a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "opmm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(opmm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_three_calls():
    names = _declared()
    for n in ("opmm_simulate", "opmm_score", "opmm_fit"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2007_09884_amd import opmm
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(opmm.lib, n), n
        assert ctypes.cast(getattr(opmm.lib, n), ctypes.c_void_p).value


def test_struct_layouts_match_header():
    from paper_2007_09884_amd import opmm
    assert opmm.SACCADE_DTYPE.itemsize == 40
    assert ctypes.sizeof(opmm.FitParams) == 36
    assert ctypes.sizeof(opmm.ServeParams) == 96 and ctypes.sizeof(opmm.NmParams) == 20
    assert ctypes.sizeof(opmm.PolishParams) == 24
    q = opmm.polish_params()
    assert (q.max_iter, q.objective, q.lambda0, q.box_frac, q.dt_ms) == (20, 0, np.float32(1e-3), 0.25, 1.0)
    p = opmm.fit_params()
    assert (p.n_cand, p.n_rounds, p.box_frac, p.w_init_frac, p.shrink, p.dt_ms, p.mode, p.tile, p.model) == \
        (4096, 1, 0.25, 1.0, 0.5, 1.0, 0, -1, 18)


def test_nominal_is_table1():
    """The library's nominal OPC (host call, no GPU) equals Table 1 as the paper prints it."""
    from paper_2007_09884_amd import opmm
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "table1_nominal.txt"))
            if not l.startswith("#")]
    nom = opmm.nominal(43.0)
    for j, (_, v) in enumerate(rows[:17]):
        assert nom[j] == np.float32(float(v))
    assert nom[17] == np.float32(37.0)


def test_tile_shapes_listed():
    from paper_2007_09884_amd import opmm
    names = opmm.tile_names()
    assert len(names) >= 4 and all(names)


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2007_09884_amd import opmm
    with pytest.raises(opmm.OpmmError):
        opmm.Context(0)
