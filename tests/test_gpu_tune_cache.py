"""The autotuner cache: a pick is filed under its batch's key, saved to a text file, loaded by a
fresh context of the same architecture, and used for tile = -1; foreign and unknown lines are
skipped, malformed ones rejected."""
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


def _fit(ctx, opmm, pos, recs, prm):
    S = recs.shape[0]
    opc = torch.zeros(S, 18, device="cuda")
    rmse = torch.zeros(S, device="cuda")
    ctx.fit(pos, recs, prm, opc, rmse)
    torch.cuda.synchronize()
    return opc.cpu().numpy(), rmse.cpu().numpy()


def test_autotune_cache_round_trip(opmm, tmp_path):
    b, traces = make_batch(32, seed=synth.BASE_SEED + 77)
    recs = records(b, opmm)
    pos = torch.from_numpy(opmm.pack_traces(traces)).cuda()
    prm = opmm.fit_params(n_cand=4096, n_rounds=2)
    a = opmm.Context(0)
    assert a.tune_cache_lookup(recs, prm) == -1
    tile = a.autotune(pos, recs, prm)
    assert 0 <= tile < len(opmm.tile_names())
    assert a.tune_cache_lookup(recs, prm) == tile
    path = tmp_path / "tune.txt"
    a.tune_cache_save(str(path))
    lines = [l.split() for l in path.read_text().splitlines() if not l.startswith("#")]
    assert len(lines) == 1 and lines[0][6] == opmm.tile_names()[tile]
    arch = lines[0][0]
    assert arch.startswith("gfx")
    # the key: mode 0, model 18, longest trace and batch size rounded up to powers of two, n_cand
    tmax = int(max(b["T"]))
    assert [int(v) for v in lines[0][1:6]] == [0, 18, 1 << (tmax - 1).bit_length(), 32, 4096]
    a.close()

    c = opmm.Context(0)
    assert c.tune_cache_lookup(recs, prm) == -1
    c.tune_cache_load(str(path))
    assert c.tune_cache_lookup(recs, prm) == tile
    # other keys are not filed: more candidates, the persistent mode, a longer batch
    assert c.tune_cache_lookup(recs, opmm.fit_params(n_cand=8192, n_rounds=2)) == -1
    assert c.tune_cache_lookup(recs, opmm.fit_params(n_cand=4096, n_rounds=2, mode=1)) == -1
    assert c.tune_cache_lookup(np.concatenate([recs, recs]), prm) == -1
    # a fit with tile = -1 runs the filed shape; results never depend on the shape
    ref = _fit(c, opmm, pos, recs, opmm.fit_params(n_cand=4096, n_rounds=2, tile=(tile + 1) % len(opmm.tile_names())))
    got = _fit(c, opmm, pos, recs, prm)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])

    # lines of another architecture and unknown shapes are skipped; a replaced key takes the new shape
    other = (tile + 1) % len(opmm.tile_names())
    p2 = tmp_path / "more.txt"
    p2.write_text("# comment\n"
                  "gfx000 0 18 128 32 4096 %s 1.0\n" % opmm.tile_names()[other] +
                  "%s 0 18 256 32 4096 no_such_shape 1.0\n" % arch +
                  "%s %s %s\n" % (arch, " ".join(lines[0][1:6]), opmm.tile_names()[other] + " 2.0"))
    c.tune_cache_load(str(p2))
    assert c.tune_cache_lookup(recs, prm) == other
    # a malformed line rejects the whole file
    p3 = tmp_path / "bad.txt"
    p3.write_text("%s 0 18 128 32 4096 %s 1.0\n%s 7 18 128 32 4096 %s 1.0\n"
                  % (arch, opmm.tile_names()[tile], arch, opmm.tile_names()[tile]))
    with pytest.raises(opmm.OpmmError):
        c.tune_cache_load(str(p3))
    assert c.tune_cache_lookup(recs, prm) == other
    with pytest.raises(opmm.OpmmError):
        c.tune_cache_load(str(tmp_path / "missing.txt"))
    c.close()
