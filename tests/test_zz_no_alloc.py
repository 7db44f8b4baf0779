"""The allocation-free fit (opmm_fit_noalloc: device scratch in a static per-device array, host
staging in a static buffer) against opmm_fit on the same inputs, through the C ABI.  The bar is bit
identity of every output: both queue the same kernels on the same records; only where the scratch
lives differs.  Two calls in a row, the second on a smaller batch, so the second reads an array that
still holds the first call's contents; per-round and persistent launches; with and without caller
round keys (without, the keys live in the static array too); and the size limits."""
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


@pytest.fixture(scope="module")
def ctx(opmm):
    c = opmm.Context(0)
    yield c
    c.close()


def run(ctx, opmm, fn, b, traces, n_cand, R, mode, ncand=None, with_keys=True):
    S = b["S"]
    recs = records(b, opmm, n_cand=ncand)
    pos = torch.from_numpy(opmm.pack_traces(traces)).cuda()
    prm = opmm.fit_params(n_cand=n_cand, n_rounds=R, mode=mode)
    opc = torch.full((S, 18), -1.0, device="cuda")
    rmse = torch.full((S,), -1.0, device="cuda")
    mae = torch.full((S,), -1.0, device="cuda")
    st = torch.full((S,), -1, dtype=torch.int32, device="cuda")
    keys = torch.zeros(R, S, dtype=torch.int64, device="cuda") if with_keys else None
    getattr(ctx, fn)(pos, recs, prm, opc, rmse, mae, st, keys)
    ctx.sync()
    out = dict(opc=opc.cpu().numpy().view(np.uint32), rmse=rmse.cpu().numpy().view(np.uint32),
               mae=mae.cpu().numpy().view(np.uint32), status=st.cpu().numpy())
    if with_keys:
        out["keys"] = keys.cpu().numpy()
    return out


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in a)


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_fit_equals_fit(ctx, opmm, mode):
    cases = [(make_batch(40, "uneven", seed=424242), 3000, 4,
              np.array([3000, 64, 5000, 1] * 10, np.int32)),
             (make_batch(7, "full", seed=515151), 1000, 3, None)]
    for with_keys in (True, False):
        for (b, traces), n, R, ncand in cases:      # second call: fewer saccades, shorter traces
            ref = run(ctx, opmm, "fit", b, traces, n, R, mode, ncand, with_keys)
            got = run(ctx, opmm, "fit_noalloc", b, traces, n, R, mode, ncand, with_keys)
            assert same(ref, got), (mode, with_keys, b["S"])
            assert np.all(ref["status"] == 0)


def test_noalloc_limits(ctx, opmm):
    maxs = 4096
    T = 2048
    # the layout of 4096 saccades of 2048 samples needs 32 MiB of projections: rejected
    recs = opmm.saccade_records([T] * maxs, 1, [10.0] * maxs, [0.0] * maxs, [43.0] * maxs,
                                np.arange(maxs, dtype=np.uint64))
    pos = torch.zeros(maxs * T, device="cuda")
    opc = torch.zeros(maxs + 1, 18, device="cuda"); rmse = torch.zeros(maxs + 1, device="cuda")
    with pytest.raises(opmm.OpmmError) as e:
        ctx.fit_noalloc(pos, recs, opmm.fit_params(), opc, rmse)
    assert e.value.code == opmm.EINVAL and "bytes of scratch" in str(e.value)
    recs = opmm.saccade_records([20] * (maxs + 1), 1, [10.0] * (maxs + 1), [0.0] * (maxs + 1),
                                [43.0] * (maxs + 1), np.arange(maxs + 1, dtype=np.uint64))
    with pytest.raises(opmm.OpmmError) as e:
        ctx.fit_noalloc(pos, recs, opmm.fit_params(), opc, rmse)
    assert e.value.code == opmm.EINVAL and "NOALLOC_MAX_S" in str(e.value)
    # after a rejection the entry point still works
    b, traces = make_batch(3, "full", seed=616161)
    assert same(run(ctx, opmm, "fit", b, traces, 500, 2, 0), run(ctx, opmm, "fit_noalloc", b, traces, 500, 2, 0))
