"""The paper's parallel Nelder-Mead on the GPU vs the oracle's serial Nelder-Mead (same Lagarias steps),
replayed decision by decision: the oracle follows the GPU's decisions and, at every iteration, also
takes its own; the two may differ only where the comparison that decided rested on values closer than
1e-6 (both choices valid there).  Following the same decisions, the two runs end at the same vertex."""
import numpy as np
import pytest

import oracle
from paper_2007_09884_amd import synth
from workload import make_batch, records

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GAP = 1e-6


@pytest.fixture(scope="module")
def opmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_09884_amd import opmm as m
    return m


@pytest.fixture(scope="module")
def ctx(opmm):
    c = opmm.Context(0)
    yield c
    c.close()


def run_nm(ctx, opmm, b, traces, prm, status=False):
    S = b["S"]
    recs = records(b, opmm)
    pos = torch.from_numpy(opmm.pack_traces(traces)).cuda()
    opc = torch.zeros(S, 18, device="cuda"); rm = torch.zeros(S, device="cuda")
    it = torch.zeros(S, dtype=torch.int32, device="cuda")
    dec = torch.full((S, max(prm.max_iter, 1)), -1, dtype=torch.int8, device="cuda")
    st = torch.full((S,), -1, dtype=torch.int32, device="cuda")
    ctx.fit_nm(pos, recs, prm, opc, rm, it, dec, st)
    torch.cuda.synchronize()
    out = (opc.cpu().numpy(), rm.cpu().numpy(), it.cpu().numpy(), dec.cpu().numpy())
    return out + (st.cpu().numpy(),) if status else out


@pytest.mark.parametrize("kind", ["tiny", "full"])
def test_nelder_mead_replays_against_oracle(ctx, opmm, kind):
    b, traces = make_batch(3, kind, seed=synth.BASE_SEED + 61)
    prm = opmm.nm_params(max_iter=120, tol_x=0.0, tol_f=0.0)
    opc, rm, it, dec = run_nm(ctx, opmm, b, traces, prm)
    assert np.all(it == 120)
    for s in range(b["S"]):
        r = oracle.nelder_mead(traces[s], b["amp"][s], b["dir_deg"][s], b["dur_ms"][s], max_iter=120, tol_x=0.0,
                               tol_f=0.0, forced=dec[s, :120])
        differ = r["own"] != dec[s, :120]
        assert np.all(r["margin"][differ] < GAP), (s, np.nonzero(differ), r["margin"][differ])
        assert np.abs(r["opc"].astype(np.float64) / opc[s] - 1).max() <= 1e-6, s
        assert abs(r["rmse"] - rm[s]) <= 1e-6 * max(1.0, r["rmse"])


def test_nelder_mead_converges_and_improves_on_nominal(ctx, opmm):
    b, traces = make_batch(4, "full", seed=synth.BASE_SEED + 71)
    prm = opmm.nm_params(max_iter=3000, tol_x=1e-4, tol_f=1e-6)
    opc, rm, it, dec = run_nm(ctx, opmm, b, traces, prm)
    for s in range(b["S"]):
        nom = oracle.nominal(b["dur_ms"][s]).astype(np.float32).astype(np.float64)
        r0, _ = oracle.cost(oracle.simulate(nom, b["amp"][s], int(b["T"][s])), traces[s], b["dir_deg"][s])
        assert rm[s] < r0
        r1, _ = oracle.cost(oracle.simulate(opc[s].astype(np.float64), b["amp"][s], int(b["T"][s])), traces[s],
                            b["dir_deg"][s])
        assert abs(r1 - rm[s]) <= 1e-6   # reported cost is the oracle's cost of the returned vertex
        assert 0 < it[s] <= 3000
        assert np.all(dec[s, :it[s]] >= 0) and np.all(dec[s, :it[s]] <= 4)


def _mixed_batch():
    """Seven saccades of both configurations (1 and 2 channels do not mix in one batch: the full ones
    only), T from 26 to 87: two tasks per wave pair saccades of different lengths, the last wave ragged."""
    return make_batch(7, "full", seed=synth.BASE_SEED + 81)


def test_nelder_mead_wave_layouts_agree(ctx, opmm):
    """One and two tasks per wave run each task's arithmetic unchanged: results, iteration counts and
    decisions are identical, with tolerances that stop tasks at different iterations."""
    b, traces = _mixed_batch()
    for tol in ((0.0, 0.0), (0.02, 5e-3)):
        outs = []
        for g in (1, 2):
            prm = opmm.nm_params(max_iter=300, tol_x=tol[0], tol_f=tol[1], tasks_per_wave=g)
            outs.append(run_nm(ctx, opmm, b, traces, prm, status=True))
        a, c = outs
        assert np.array_equal(a[0].view(np.uint32), c[0].view(np.uint32)) and np.array_equal(a[1], c[1]), tol
        assert np.array_equal(a[2], c[2]) and np.array_equal(a[3], c[3]) and np.all(a[4] == 0), tol
    assert len(set(a[2].tolist())) > 1   # the tasks stopped at different iterations


def test_nelder_mead_time_bound(ctx, opmm):
    """The time bound (Section 3.3's exit criteria include a time limit): a budget of the shortest
    measurable time stops every task at its first exit test with OPMM_ST_DEADLINE, returning the best
    vertex of the initial simplex (the oracle's, at zero iterations) and its cost; a generous budget
    changes nothing."""
    b, traces = _mixed_batch()
    for g in (1, 2):
        opc, rm, it, dec, st = run_nm(ctx, opmm, b, traces,
                                      opmm.nm_params(max_iter=500, max_ms=1e-6, tasks_per_wave=g), status=True)
        assert np.all(it == 0) and np.all(st == opmm.ST_DEADLINE), (it, st)
        for s in range(b["S"]):
            r = oracle.nelder_mead(traces[s], b["amp"][s], b["dir_deg"][s], b["dur_ms"][s], max_iter=0)
            assert np.abs(r["opc"].astype(np.float64) / opc[s] - 1).max() <= 1e-6, s
            assert abs(r["rmse"] - rm[s]) <= 1e-6 * max(1.0, r["rmse"]), s
    free = run_nm(ctx, opmm, b, traces, opmm.nm_params(max_iter=100, tol_x=0.0, tol_f=0.0), status=True)
    slow = run_nm(ctx, opmm, b, traces, opmm.nm_params(max_iter=100, tol_x=0.0, tol_f=0.0, max_ms=1e5), status=True)
    assert all(np.array_equal(x, y) for x, y in zip(free, slow)) and np.all(free[4] == 0)
