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
    assert ctypes.sizeof(opmm.FitParams) == 44
    assert ctypes.sizeof(opmm.ServeParams) == 120 and ctypes.sizeof(opmm.NmParams) == 28
    sv = opmm.serve_params()
    assert (sv.max_slots, sv.max_T, sv.polish_iter, sv.rounds_per_step) == (4096, 160, 0, 16)
    n = opmm.nm_params()
    assert (n.max_iter, n.tol_x, n.tol_f, n.box_frac, n.dt_ms, n.max_ms, n.tasks_per_wave) == \
        (500, np.float32(1e-4), np.float32(1e-6), 0.25, 1.0, 0.0, 0)
    assert ctypes.sizeof(opmm.PolishParams) == 24
    q = opmm.polish_params()
    assert (q.max_iter, q.objective, q.lambda0, q.box_frac, q.dt_ms) == (20, 0, np.float32(1e-3), 0.25, 1.0)
    p = opmm.fit_params()
    assert (p.n_cand, p.n_rounds, p.box_frac, p.w_init_frac, p.shrink, p.dt_ms, p.mode, p.tile, p.model,
            p.screen_rounds, p.screen_tol) == (4096, 1, 0.25, 1.0, 0.5, 1.0, 0, -1, 18, 0, np.float32(5e-5))


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


def test_result_file_matches_the_papers_format(tmp_path):
    """The result writer reproduces the column set of the paper's example output (Fig. 4), reads the
    printed rows back into Table 1 order, and writes them again digit for digit."""
    from paper_2007_09884_amd import report
    lines = [l for l in open(os.path.join(os.path.dirname(__file__), "golden", "fig4_output.txt"))
             if not l.startswith("#")]
    assert lines[0].strip().split(",") == report.COLUMNS
    src = tmp_path / "fig4.csv"
    src.write_text("".join(lines))
    opc, err, chk = report.read_csv(str(src))
    assert opc.shape == (2, 18)
    # Table 1 positions: K_SE_AG, N_C_AG (tension slope), B_P (passive viscosity), J (inertia), PW
    assert opc[0, 0] == 25.0 and opc[0, 7] == 8.0 and opc[0, 6] == 0.006063 and opc[0, 9] == 0.000043
    assert opc[1, 17] == 7.316801 and opc[1, 15] == 126.041275
    assert list(err) == [10.701933, 1.115680] and list(chk) == [10.701933, 1.115681]
    out = tmp_path / "again.csv"
    report.write_csv(str(out), opc, err, chk)
    again = out.read_text().splitlines()
    assert again[0] == lines[0].strip()
    assert again[2] == lines[2].strip()   # every printed value has six decimals in row 2
    # a result without the serial re-check leaves that column empty
    report.write_csv(str(out), opc[:1], err[:1])
    assert out.read_text().splitlines()[1].split(",")[2] == ""


def test_null_handles_are_rejected():
    """Every call that takes a context, surrogate, plan or server handle rejects a null one with
    OPMM_EINVAL before touching anything (no GPU needed); destroy calls accept null."""
    from paper_2007_09884_amd import opmm
    seen = 0
    for n in _declared():
        fn = getattr(opmm.lib, n)
        a = fn.argtypes
        if not a or a[0] is not ctypes.c_void_p:
            continue
        vals = [0.0 if t in (ctypes.c_float, ctypes.c_double) else
                0 if t in (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64) else None
                for t in a]
        r = fn(*vals)
        if n.endswith("_destroy"):
            assert r == 0, n
        elif n == "opmm_last_error":
            assert r
        elif n == "opmm_server_slots":
            assert r == 0
        else:
            assert r == -1, (n, r)
        seen += 1
    assert seen >= 35
