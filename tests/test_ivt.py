"""I-VT extraction: the oracle's plain-loop reference pinned on hand-built streams (CPU), and the GPU
kernels against it on a synthetic recording made of fixations and plant-simulated saccades (GPU)."""
import numpy as np
import pytest

import oracle


def synthetic_stream(rng, n_sacc=12, noise=0.003):
    """Fixations (100-300 ms, tiny noise) joined by saccades simulated by the plant."""
    pos = np.zeros(2)
    parts, planted = [], []
    t = 0
    for i in range(n_sacc):
        fix = int(rng.integers(100, 300))
        parts.append(np.tile(pos, (fix, 1)))
        t += fix
        amp = rng.uniform(3, 20)
        phi = rng.uniform(0, 360)
        dur = 2.2 * amp + 21
        T = int(np.ceil(dur)) + 30
        p = oracle.nominal(dur) * rng.uniform(0.9, 1.1, 18)
        th = oracle.simulate(p, amp, T)
        u = np.array([np.cos(np.radians(phi)), np.sin(np.radians(phi))])
        parts.append(pos + th[:, None] * u[None, :])
        planted.append((t, amp, phi))
        t += T
        pos = pos + amp * u
    parts.append(np.tile(pos, (150, 1)))
    g = np.concatenate(parts)
    g = g + noise * rng.standard_normal(g.shape)
    return g.astype(np.float32), planted


def test_ivt_reference_by_hand():
    g = np.zeros((12, 2), np.float32)
    g[4] = [0.5, 0.0]             # fast at samples 4, 5, 6 (>= 500 deg/s), slow elsewhere
    g[5] = [1.0, 0.0]
    g[6:] = [1.5, 0.5]
    out = oracle.ivt(g, vel_thresh=30.0, min_dur=0.0)
    assert len(out) == 1
    s = out[0]
    assert s["start"] == 3 and s["T"] == 4      # samples 3 (fixation) .. 6
    assert abs(s["amp"] - np.hypot(1.5, 0.5)) < 1e-6 and abs(s["dir"] - np.degrees(np.arctan2(0.5, 1.5))) < 1e-4
    assert np.array_equal(s["trace"][0], [0, 0]) and np.array_equal(s["trace"][-1], [1.5, 0.5])
    assert oracle.ivt(g, vel_thresh=30.0, min_dur=6.0) == []   # 3 ms run dropped


def test_ivt_reference_finds_planted_saccades():
    rng = np.random.default_rng(3)
    g, planted = synthetic_stream(rng)
    out = oracle.ivt(g, vel_thresh=30.0, min_dur=6.0)
    assert len(out) == len(planted)
    for s, (t0, amp, phi) in zip(out, planted):
        assert t0 <= s["start"] <= t0 + 15                          # onset: first fast sample
        assert s["amp"] < amp + 0.05                                # cut when the eye slows below threshold
        assert abs((s["dir"] - phi + 180) % 360 - 180) < 2.0


@pytest.mark.gpu
def test_ivt_gpu_matches_reference():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_09884_amd import opmm
    ctx = opmm.Context(0)
    rng = np.random.default_rng(4)
    g, planted = synthetic_stream(rng, n_sacc=40)
    ref = oracle.ivt(g, vel_thresh=30.0, min_dur=6.0)
    pos = torch.zeros(200000, device="cuda")
    recs, src = ctx.ivt_extract(torch.from_numpy(g).cuda(), pos, vel_thresh=30.0, min_dur=6.0, max_out=100)
    torch.cuda.synchronize()
    assert len(recs) == len(ref) == len(planted)
    P = pos.cpu().numpy()
    for r, s, k in zip(ref, recs, src):
        assert k == r["start"] and s["T"] == r["T"] and s["C"] == 2
        assert abs(s["amp_deg"] - r["amp"]) <= 1e-5 * max(1, r["amp"])
        assert abs((s["dir_deg"] - r["dir"] + 180) % 360 - 180) <= 1e-3
        tr = P[s["pos_offset"]:s["pos_offset"] + 2 * s["T"]].reshape(-1, 2)
        assert np.array_equal(tr, r["trace"])
        assert s["dur_ms"] == np.float32(s["T"] - 1)
    # the extracted saccades feed the fit directly
    opc = torch.zeros(len(recs), 18, device="cuda"); rm = torch.zeros(len(recs), device="cuda")
    ctx.fit(pos, recs, opmm.fit_params(n_cand=2048, n_rounds=3), opc, rm)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(rm.cpu().numpy()))
    ctx.close()


@pytest.mark.gpu
def test_ivt_gpu_truncation_and_edges():
    """max_out and the trace capacity cut the output in stream order; a stream with no fast sample
    or shorter than two samples gives nothing; bad arguments are rejected."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_09884_amd import opmm
    ctx = opmm.Context(0)
    rng = np.random.default_rng(6)
    g, planted = synthetic_stream(rng, n_sacc=10)
    ref = oracle.ivt(g, vel_thresh=30.0, min_dur=6.0)
    d = torch.from_numpy(g).cuda()
    pos = torch.zeros(100000, device="cuda")
    recs, src = ctx.ivt_extract(d, pos, max_out=4)
    assert len(recs) == 4 and list(src) == [r["start"] for r in ref[:4]]
    cap = 2 * sum(r["T"] for r in ref[:3]) + 1          # room for three traces, not four
    small = torch.zeros(cap, device="cuda")
    recs, src = ctx.ivt_extract(d, small, max_out=100)
    assert len(recs) == 3 and list(src) == [r["start"] for r in ref[:3]]
    still = torch.zeros(500, 2, device="cuda")
    assert len(ctx.ivt_extract(still, pos)[0]) == 0
    assert len(ctx.ivt_extract(still[:1], pos)[0]) == 0
    with pytest.raises(opmm.OpmmError):
        ctx.ivt_extract(d, pos, dt_ms=0.0)
    ctx.close()
