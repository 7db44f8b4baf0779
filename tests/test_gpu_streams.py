"""Calls on one context, plan or surrogate from two streams.  The library orders them itself (each
call records an event on its stream; a call on another stream first waits for it), so interleaved
calls give, bit for bit, what the same calls give one after another on one stream.

The two batches of a pair have the same shape (same trace lengths and candidate counts; different
noise and candidate-stream seeds), so both calls' records hold the same offsets and sizes."""
import numpy as np
import pytest

from oracle import mlp_ref
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


def _pair(opmm, S=64):
    """Two batches of one shape: (pos, recs) x 2."""
    seed = synth.BASE_SEED + 4242
    b1, tr1 = make_batch(S, seed=seed)
    b2, tr2 = make_batch(S, seed=seed, sigma=0.3)
    assert list(b1["T"]) == list(b2["T"])
    r1 = records(b1, opmm)
    r2 = records(b2, opmm)
    r2["seed"] = r2["seed"] + np.uint64(977)
    p1 = torch.from_numpy(opmm.pack_traces(tr1)).cuda()
    p2 = torch.from_numpy(opmm.pack_traces(tr2)).cuda()
    return (p1, r1), (p2, r2)


def _outs(S, R):
    return dict(opc=torch.zeros(S, 18, device="cuda"), rmse=torch.zeros(S, device="cuda"),
                mae=torch.zeros(S, device="cuda"), st=torch.zeros(S, dtype=torch.int32, device="cuda"),
                keys=torch.zeros(R, S, dtype=torch.int64, device="cuda"))


def _fit(ctx, pos, recs, prm, o, stream):
    ctx.fit(pos, recs, prm, o["opc"], o["rmse"], o["mae"], o["st"], o["keys"], stream=stream)


def _host(o):
    return {k: v.cpu().numpy() for k, v in o.items()}


def _same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k]), (what, k)


def test_fits_on_two_streams_match_one_stream(ctx, opmm):
    S, R = 64, 10
    (p1, r1), (p2, r2) = _pair(opmm, S)
    prm = opmm.fit_params(n_cand=65536, n_rounds=R)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    ref1, ref2 = _outs(S, R), _outs(S, R)
    _fit(ctx, p1, r1, prm, ref1, sa)
    sa.synchronize()
    _fit(ctx, p2, r2, prm, ref2, sa)
    sa.synchronize()
    h1, h2 = _host(ref1), _host(ref2)
    assert not np.array_equal(h1["opc"], h2["opc"])
    for rep in range(3):
        o1, o2 = _outs(S, R), _outs(S, R)
        torch.cuda.synchronize()
        first, second = (sa, sb) if rep % 2 == 0 else (sb, sa)
        print("interleaved fits, repeat", rep, flush=True)
        _fit(ctx, p1, r1, prm, o1, first)
        _fit(ctx, p2, r2, prm, o2, second)
        ctx.sync(first)
        ctx.sync(second)
        _same(_host(o1), h1, ("first", rep))
        _same(_host(o2), h2, ("second", rep))


def test_plan_launches_on_two_streams(ctx, opmm):
    S, R = 64, 10
    (p1, r1), _ = _pair(opmm, S)
    prm = opmm.fit_params(n_cand=65536, n_rounds=R, mode=1)
    o = _outs(S, R)
    plan = ctx.plan(p1, r1, prm, o["opc"], o["rmse"], o["mae"], o["st"], o["keys"])
    torch.cuda.synchronize()
    ref = _host(o)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for k in o.values():
        k.zero_()
    torch.cuda.synchronize()
    plan.launch(sa)
    plan.launch(sb)
    plan.launch(sa)
    ctx.sync(sa)
    ctx.sync(sb)
    _same(_host(o), ref, "plan")
    plan.close()


def test_surrogate_calls_on_two_streams(ctx, opmm):
    sg = opmm.Surrogate(ctx, init_seed=5)
    B = 4096
    rng = np.random.default_rng(3)
    f1 = torch.from_numpy(mlp_ref.bf16_bits(rng.normal(0, 0.5, (B, 256))).view(np.int16)).cuda()
    f2 = torch.from_numpy(mlp_ref.bf16_bits(rng.normal(0, 0.5, (B, 256))).view(np.int16)).cuda()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    r1, r2 = torch.zeros(B, 18, device="cuda"), torch.zeros(B, 18, device="cuda")
    torch.cuda.synchronize()
    sg.forward(f1, r1, stream=sa)
    sa.synchronize()
    sg.forward(f2, r2, stream=sa)
    sa.synchronize()
    h1, h2 = r1.cpu().numpy(), r2.cpu().numpy()
    for rep in range(3):
        o1, o2 = torch.zeros_like(r1), torch.zeros_like(r2)
        torch.cuda.synchronize()
        sg.forward(f1, o1, stream=sa)
        sg.forward(f2, o2, stream=sb)
        sb.synchronize()
        sa.synchronize()
        assert np.array_equal(o1.cpu().numpy(), h1), rep
        assert np.array_equal(o2.cpu().numpy(), h2), rep
    sg.close()
