"""Kernel timing (opmm_kernel_timing_enable / _read): a directly queued fit records one event pair
per search-kernel launch, per kind; a plan's graph launches record none; reads clear what they return;
timing off records nothing; bad arguments are rejected.  Timing changes no result."""
import numpy as np
import pytest

from workload import make_batch, records

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def opmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_09884_amd import opmm as m
    return m


def run(ctx, opmm, b, traces, prm, plan=False):
    S, R = b["S"], prm.n_rounds
    recs = records(b, opmm)
    pos = torch.from_numpy(opmm.pack_traces(traces)).cuda()
    opc, rmse, mae = (torch.zeros(S, 18, device="cuda"), torch.zeros(S, device="cuda"),
                      torch.zeros(S, device="cuda"))
    status = torch.zeros(S, dtype=torch.int32, device="cuda")
    keys = torch.zeros(R, S, dtype=torch.int64, device="cuda")
    if plan:
        pl = ctx.plan(pos, recs, prm, opc, rmse, mae, status, keys)
        pl.launch()
        ctx.sync()
        pl.close()
    else:
        ctx.fit(pos, recs, prm, opc, rmse, mae, status, keys)
        ctx.sync()
    return opc.cpu().numpy(), keys.cpu().numpy()


def counts(ctx, opmm):
    return {k: ctx.kernel_times(k) for k in (opmm.KERNEL_ROUND, opmm.KERNEL_SCREEN, opmm.KERNEL_VERIFY,
                                             opmm.KERNEL_PERSISTENT)}


def test_kernel_timing_counts_each_launch(opmm):
    b, traces = make_batch(8, "full")
    prm = opmm.fit_params(n_cand=4096, n_rounds=5, screen_rounds=3)
    ctx = opmm.Context(0)
    try:
        ref = run(ctx, opmm, b, traces, prm)
        assert all(v == (0.0, 0) for v in counts(ctx, opmm).values())  # off by default
        ctx.kernel_timing(True)
        got = run(ctx, opmm, b, traces, prm)
        got2 = run(ctx, opmm, b, traces, prm)
        for a, r in zip(got + got2, ref + ref):
            assert np.array_equal(a, r)
        c = counts(ctx, opmm)
        assert c[opmm.KERNEL_SCREEN][1] == 6 and c[opmm.KERNEL_VERIFY][1] == 6
        assert c[opmm.KERNEL_ROUND][1] == 4 and c[opmm.KERNEL_PERSISTENT][1] == 0
        for k in (opmm.KERNEL_SCREEN, opmm.KERNEL_VERIFY, opmm.KERNEL_ROUND):
            assert c[k][0] > 0.0
        assert all(v == (0.0, 0) for v in counts(ctx, opmm).values())  # a read clears
        # persistent mode: one launch per fit
        run(ctx, opmm, b, traces, opmm.fit_params(n_cand=4096, n_rounds=5, mode=opmm.FIT_PERSISTENT))
        assert ctx.kernel_times(opmm.KERNEL_PERSISTENT)[1] == 1
        # a plan: its creation runs the fit once uncaptured (recorded), its graph launches record nothing
        run(ctx, opmm, b, traces, prm, plan=True)
        c = counts(ctx, opmm)
        assert (c[opmm.KERNEL_SCREEN][1], c[opmm.KERNEL_VERIFY][1], c[opmm.KERNEL_ROUND][1]) == (3, 3, 2)
        # switched off: nothing recorded
        ctx.kernel_timing(False)
        run(ctx, opmm, b, traces, prm)
        assert all(v[1] == 0 for v in counts(ctx, opmm).values())
        with pytest.raises(opmm.OpmmError):
            ctx.kernel_times(opmm.KERNEL_PERSISTENT + 1)
        with pytest.raises(opmm.OpmmError):
            ctx.kernel_times(-1)
    finally:
        ctx.close()
