"""Continuous-batching server on the GPU, through the C ABI: each result is the same alone (opmm_fit
/ opmm_fit_learned on that saccade only) and in the mix (admitted at different times, sharing
launches with other requests at other rounds); admission is bounded by the HBM budget."""
import numpy as np
import pytest

from paper_2007_09884_amd import synth
from workload import make_batch, records

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


def stream_through(server, b, traces, recs, waves=(4, 3, 5)):
    """Submit in waves with steps in between, so requests share launches at different rounds."""
    n, i, out = b["S"], 0, []
    for w in waves:
        for k in range(i, min(n, i + w)):
            server.submit(traces[k], recs[k])
        i += w
        server.step()
        out.append(server.poll())
    for k in range(i, n):
        server.submit(traces[k], recs[k])
    for _ in range(200):
        if server.stats()["completed"] == n:
            break
        server.step()
        out.append(server.poll())
    out.append(server.poll())
    res = {k: np.concatenate([o[k] for o in out]) for k in out[0]}
    order = np.argsort(res["id"])
    return {k: v[order] for k, v in res.items()}


@pytest.mark.parametrize("rounds_per_step", [1, 16])
def test_plain_server_results_equal_fit_alone(ctx, opmm, rounds_per_step):
    """Results equal opmm_fit on each saccade alone, whether a step runs one round (rounds_per_step
    1) or, while the device would idle, several (the default 16: a light load like this one then
    finishes each search in the step that admitted it)."""
    b, traces = make_batch(14, "full", seed=synth.BASE_SEED + 31)
    recs = records(b, opmm)
    recs["pos_offset"] = 0
    prm = opmm.serve_params(max_slots=6, rounds_per_step=rounds_per_step)
    prm.plain.n_cand = 3000
    prm.plain.n_rounds = 4
    sv = opmm.Server(ctx, prm)
    res = stream_through(sv, b, traces, recs)
    steps = sv.stats()["steps"]
    assert len(res["id"]) == b["S"] and np.all(res["status"] == 0)
    assert np.all(res["t_done"] >= res["t_arrival"])
    fp = opmm.fit_params(n_cand=3000, n_rounds=4)
    for s in range(b["S"]):
        opc = torch.zeros(1, 18, device="cuda"); rm = torch.zeros(1, device="cuda")
        ctx.fit(torch.from_numpy(traces[s].reshape(-1)).cuda(), recs[s:s + 1], fp, opc, rm)
        torch.cuda.synchronize()
        assert np.array_equal(opc.cpu().numpy()[0].view(np.uint32), res["opc"][s].view(np.uint32)), s
        assert rm.cpu().numpy()[0] == res["rmse"][s]
    st = sv.stats()
    assert st["completed"] == b["S"] and st["busy"] == 0 and st["pending"] == 0
    # 14 requests x 4 rounds through at most 6 slots take at least 10 steps at one round per step;
    # with several, each search ends in the step that admitted it (four submission waves)
    assert steps >= 10 if rounds_per_step == 1 else steps <= 6, steps
    sv.close()
    for bad in (0, 65):
        with pytest.raises(opmm.OpmmError):
            opmm.Server(ctx, opmm.serve_params(rounds_per_step=bad))


def test_polished_server_results_equal_fit_and_polish_alone(ctx, opmm):
    """With polish_iter > 0 every finished search is polished on the server's polish streams (up to
    three batches in flight; 24 requests through 4 slots keep them full): the result equals
    opmm_fit followed by opmm_polish on that saccade alone."""
    b, traces = make_batch(24, "full", seed=synth.BASE_SEED + 35)
    recs = records(b, opmm)
    recs["pos_offset"] = 0
    prm = opmm.serve_params(max_slots=4, polish_iter=3)
    prm.plain.n_cand = 2048
    prm.plain.n_rounds = 3
    sv = opmm.Server(ctx, prm)
    res = stream_through(sv, b, traces, recs, waves=(3, 2, 5, 4))
    assert len(res["id"]) == b["S"]
    fp = opmm.fit_params(n_cand=2048, n_rounds=3)
    pp = opmm.polish_params(max_iter=3)
    for s in range(b["S"]):
        pos = torch.from_numpy(traces[s].reshape(-1)).cuda()
        opc = torch.zeros(1, 18, device="cuda"); rm = torch.zeros(1, device="cuda")
        ctx.fit(pos, recs[s:s + 1], fp, opc, rm)
        rm0 = float(rm.cpu()[0])
        ctx.polish(pos, recs[s:s + 1], pp, opc, rm)
        torch.cuda.synchronize()
        assert np.array_equal(opc.cpu().numpy()[0].view(np.uint32), res["opc"][s].view(np.uint32)), s
        assert rm.cpu().numpy()[0] == res["rmse"][s] and res["rmse"][s] <= rm0 * (1 + 1e-6)
    sv.close()
    with pytest.raises(opmm.OpmmError):
        opmm.Server(ctx, opmm.serve_params(polish_iter=-1))


def test_learned_server_results_equal_learned_fit_alone(ctx, opmm):
    sg = opmm.Surrogate(ctx, init_seed=9)
    sg.train(data_seed=5, batch=2048, n_steps=150)
    b, traces = make_batch(10, "full", seed=synth.BASE_SEED + 41)
    recs = records(b, opmm)
    recs["pos_offset"] = 0
    for thr in (1e9, 0.0):   # never / always fall back
        prm = opmm.serve_params(max_slots=4, fallback_rmse=thr)
        prm.plain.n_cand, prm.plain.n_rounds = 2048, 3
        prm.seeded.n_cand, prm.seeded.n_rounds = 1024, 3
        sv = opmm.Server(ctx, prm, sg)
        res = stream_through(sv, b, traces, recs, waves=(3, 2))
        for s in range(b["S"]):
            opc = torch.zeros(1, 18, device="cuda"); rm = torch.zeros(1, device="cuda")
            st = torch.zeros(1, dtype=torch.int32, device="cuda")
            sg.fit(torch.from_numpy(traces[s].reshape(-1)).cuda(), recs[s:s + 1], prm.seeded, prm.plain, thr,
                   opc, rm, st)
            torch.cuda.synchronize()
            assert np.array_equal(opc.cpu().numpy()[0].view(np.uint32), res["opc"][s].view(np.uint32)), (thr, s)
            assert rm.cpu().numpy()[0] == res["rmse"][s]
            assert st.cpu().numpy()[0] == res["status"][s]
        assert sv.stats()["fallbacks"] == (b["S"] if thr == 0.0 else 0)
        sv.close()
    sg.close()



def test_learned_polished_server_with_fallback(ctx, opmm):
    """Learned seed, polish and forced fallback together (the polish runs on the server's second
    stream and its results are taken in a later step): each result equals the seeded refine and
    the plain search, each polished alone, the lower-RMSE one kept."""
    sg = opmm.Surrogate(ctx, init_seed=9)
    sg.train(data_seed=5, batch=2048, n_steps=150)
    b, traces = make_batch(8, "full", seed=synth.BASE_SEED + 43)
    recs = records(b, opmm)
    recs["pos_offset"] = 0
    prm = opmm.serve_params(max_slots=4, fallback_rmse=0.0, polish_iter=3)
    prm.plain.n_cand, prm.plain.n_rounds = 2048, 3
    prm.seeded.n_cand, prm.seeded.n_rounds = 1024, 3
    sv = opmm.Server(ctx, prm, sg)
    res = stream_through(sv, b, traces, recs, waves=(3, 2))
    assert len(res["id"]) == b["S"]
    pp = opmm.polish_params(max_iter=3)
    for s in range(b["S"]):
        pos = torch.from_numpy(traces[s].reshape(-1)).cuda()
        seed = torch.zeros(1, 18, device="cuda")
        sg.predict(pos, recs[s:s + 1], seed, dt_ms=prm.seeded.dt_ms, box_frac=prm.seeded.box_frac)
        o1 = torch.zeros(1, 18, device="cuda"); r1 = torch.zeros(1, device="cuda")
        ctx.fit(pos, recs[s:s + 1], prm.seeded, o1, r1, seed_opc=seed)
        ctx.polish(pos, recs[s:s + 1], pp, o1, r1)
        o2 = torch.zeros(1, 18, device="cuda"); r2 = torch.zeros(1, device="cuda")
        ctx.fit(pos, recs[s:s + 1], prm.plain, o2, r2)
        ctx.polish(pos, recs[s:s + 1], pp, o2, r2)
        torch.cuda.synchronize()
        r1v, r2v = r1.cpu().numpy()[0], r2.cpu().numpy()[0]
        want = (o1 if r1v <= r2v else o2).cpu().numpy()[0]
        assert np.array_equal(want.view(np.uint32), res["opc"][s].view(np.uint32)), s
        assert res["rmse"][s] == min(r1v, r2v), s
        assert res["status"][s] & opmm.ST_FALLBACK, s
    assert sv.stats()["fallbacks"] == b["S"]
    sv.close()
    sg.close()

def test_admission_is_bounded_by_the_hbm_budget(ctx, opmm):
    prm = opmm.serve_params(max_slots=1000, hbm_budget_bytes=3 * 2800)
    prm.plain.n_cand, prm.plain.n_rounds = 512, 2
    sv = opmm.Server(ctx, prm)
    assert sv.slots == 3
    b, traces = make_batch(9, "full", seed=synth.BASE_SEED + 51)
    recs = records(b, opmm)
    recs["pos_offset"] = 0
    pos = np.concatenate([t.reshape(-1) for t in traces])
    recs2 = records(b, opmm)
    ids = sv.submit_many(pos, recs2, np.full(9, sv.now()))
    assert list(ids) == list(range(9))
    sv.step()
    st = sv.stats()
    # three slots: three requests admitted (a light step may already finish them), the rest wait for
    # memory, nothing fails
    assert st["busy"] + st["completed"] == 3 and st["pending"] == 6
    for _ in range(50):
        if sv.stats()["completed"] == 9:
            break
        sv.step()
    assert sv.stats()["completed"] == 9
    assert len(sv.poll()["id"]) == 9
    with pytest.raises(opmm.OpmmError) as e:   # longer than max_T
        sv.submit(np.zeros((prm.max_T + 1, 2), np.float32),
                  opmm.saccade_records([prm.max_T + 1], 2, [10.0], [0.0], [43.0], [1]))
    assert e.value.code == opmm.EINVAL
    sv.close()
    with pytest.raises(opmm.OpmmError):
        opmm.Server(ctx, opmm.serve_params(hbm_budget_bytes=100))
