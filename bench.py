"""Benchmark: OPC estimation on one MI355X.

Workload (the full-estimation configuration): 256 synthetic 2-D saccades,
amplitudes U[2, 30] deg, directions U[0, 360), durations from the main
sequence D = 2.2 ms/deg * A + 21 ms sampled at 1 kHz (T = ceil(D)), traces made
from true OPCs = nominal * U[0.8, 1.2] plus N(0, 0.05^2) deg noise.  A step is
one whole estimation of the batch: 65536 candidates per saccade per round, 10
rounds with the box halving each round, argmin, final report -- the fused
kernels of libopmm, launched as one captured HIP graph.  By default the tile
shape is autotuned for both launch modes (one kernel per round, or one
persistent work-queue kernel for all rounds) and the faster is timed.  Inputs
are resident in HBM before timing starts.

Prints one JSON line.  value = candidate simulations per second for the whole
job; saccades fitted per second is reported beside it.
"""
import argparse
import gc
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_CAND_SAMPLE = 54  # algorithmic work of one recurrence step + fused squared residual
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12  # 256 CU x 4 SIMD x 16 lanes x FMA x 2.4 GHz: v_fma_f64 or non-packed v_fma_f32
PUBLISHED_FP32_PEAK = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--saccades", type=int, default=256)
    ap.add_argument("--n-cand", type=int, default=65536)
    ap.add_argument("--rounds", type=int, default=10)
    ap.add_argument("--mode", choices=["auto", "persistent", "rounds"], default="rounds",
                    help="auto: autotune the tile for both launch modes and keep the faster")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--screen-rounds", type=int, default=8,
                    help="rounds screened in FP32 with the FP64 argmin of the candidates within --screen-tol "
                         "(per-round mode; results equal the FP64-only fit, which a side leg times); 0: FP64 only")
    ap.add_argument("--screen-tol", type=float, default=5e-5, help="screening tolerance, deg of RMSE")
    ap.add_argument("--no-fp64-leg", action="store_true",
                    help="skip the side leg that times the same fit with every round in FP64")
    ap.add_argument("--tile", type=int, default=-1, help="kernel shape index; -1 library default, -2 autotune")
    ap.add_argument("--no-autotune-leg", action="store_true",
                    help="skip the side leg that autotunes both launch modes and times their picks")
    ap.add_argument("--cpu-seconds", type=float, default=16.0, help="target length of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--train-saccades", type=int, default=10_000_000)
    ap.add_argument("--heldout", type=int, default=4096)
    ap.add_argument("--seed-cand", type=int, default=1024)
    ap.add_argument("--seed-rounds", type=int, default=3)
    ap.add_argument("--seed-width", type=float, default=0.25, help="round-0 half-width / box half-width")
    ap.add_argument("--polish-iter", type=int, default=4, help="Levenberg-Marquardt iterations after the seeded refine")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-uneven", action="store_true", help="skip the batched-uneven (persistent launch) leg")
    ap.add_argument("--no-nm", action="store_true")
    ap.add_argument("--no-ivt", action="store_true", help="skip the I-VT leg (gaze stream -> saccade records and traces)")
    ap.add_argument("--ivt-saccades", type=int, default=2000)
    ap.add_argument("--no-model9", action="store_true", help="skip the 9-parameter model leg")
    ap.add_argument("--no-tiny", action="store_true", help="skip the tiny-configuration latency leg")
    ap.add_argument("--report-csv", default=None,
                    help="also write the batch's results in the paper's output format (Fig. 4) to this path")
    ap.add_argument("--nm-iter", type=int, default=2000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 512 MiB device-to-device copy 3 times (calibrates HBM byte counters)")
    ap.add_argument("--serve-rates", default="2000,5000,10000,20000,50000")
    ap.add_argument("--serve-polish", type=int, default=4,
                    help="polish iterations per served request in the extra polished-serving line (0: skip it)")
    ap.add_argument("--serve-seconds", type=float, default=1.0, help="arrival window per rate")
    ap.add_argument("--serve-long-rate", type=float, default=50000.0,
                    help="rate of the one long serving window (the serving configuration's 60 s)")
    ap.add_argument("--serve-long-seconds", type=float, default=60.0, help="0 skips the long window")
    return ap.parse_args()


# The paper's own figures (Section 4.2 and its performance table; hardware from the test-system
# figure): its parallel Nelder-Mead on a private recorded dataset, so context, not a target.
PAPER_FIGURES = {
    "source": "Section 4.2, performance table; test-system figure",
    "workload": "about 60,000 saccade simulations by the paper's Nelder-Mead estimator on recorded saccades",
    "matlab_serial": {"runtime_s": 832.8, "throughput_per_s": 9.22,
                      "hardware": "Intel Xeon Silver 4116 @ 2.10 GHz (Dell R740), MATLAB"},
    "cuda": {"runtime_s": 42.6, "throughput_per_s": 464.61,
             "hardware": "NVIDIA Tesla T4 (named TU102 in the text), CUDA 10.1"},
    "unit": "simulations/s as printed (the text also calls them samples/second)",
}

# multiply-adds per sample of the 256-512-512-256-18 network: all four layers (forward, weight
# gradients) and the input gradients of layers 1-3
MLP_MACS = 256 * 512 + 512 * 512 + 512 * 256 + 256 * 18
MLP_DX_MACS = 512 * 512 + 512 * 256 + 256 * 18
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak

KERNEL_SOURCES = ("paper_2007_09884_amd/csrc/plant.hpp", "paper_2007_09884_amd/csrc/opmm.hip",
                  "paper_2007_09884_amd/csrc/runtime.hpp")


def sources_digest():
    """SHA-256 of the kernel sources with their comments removed: a counter summary stays valid across
    comment edits and goes stale with any change to the code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(text.encode())
    return h.hexdigest()


def executed_fig(flop_per_launch, launch_ms, peak):
    """Executed FLOP/s of a kernel (the VALU's own count from the profile, over this run's launch time)."""
    if flop_per_launch is None:
        return None
    t = flop_per_launch / (launch_ms * 1e-3) / 1e12
    return {"flop_per_launch": flop_per_launch, "tflops": t, "frac": t / peak,
            "source": "the VALU's own FLOP count: (SQ_INSTS_VALU_FLOPS_FP32 + _FP64) x 64 lanes x active-lane "
                      "share (rocprofv3 summary in profiles/)"}


def profiled_value(key, kernel, tile_name):
    """A per-launch figure of `kernel` from the committed rocprofv3 counter summaries (a `key=value
    kernel=.. tile=.. sources_sha256=..` line), if one was taken on the same kernel and tile shape from
    the current kernel sources; else None."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        for line in open(path):
            if line.startswith(key + "="):
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                if (kv.get("kernel") == kernel and kv.get("tile") == tile_name
                        and kv.get("sources_sha256") == sources_digest()):
                    return int(line.split()[0].split("=")[1])
    return None


def gpu_targets(ctx, opmm, torch, b):
    """Synthetic recorded traces: the plant (opmm_simulate) driven by the true OPC, projected on the
    direction, plus the drawn noise; FP32, packed [T_i][C] back to back on the device (C = 1: the
    horizontal channel only)."""
    S = b["S"]
    amp = np.asarray(b["amp"], np.float32)
    dur = np.asarray(b["dur_ms"], np.float32)
    true = np.stack([opmm.nominal(float(d)) for d in dur]) * b["mult"].astype(np.float32)
    Tmax = int(b["T"].max())
    theta = torch.zeros(S, Tmax, device="cuda")
    ctx.simulate(torch.from_numpy(true.astype(np.float32)).cuda(), torch.from_numpy(amp).cuda(), Tmax, theta)
    phi = np.deg2rad(np.asarray(b["dir_deg"], np.float32).astype(np.float64))
    parts = []
    for s in range(S):
        T = int(b["T"][s])
        u = torch.tensor([math.cos(phi[s]), math.sin(phi[s])][:b["C"]], dtype=torch.float32, device="cuda")
        z = torch.from_numpy(b["noise"][s].astype(np.float32)).cuda()
        parts.append((theta[s, :T, None] * u[None, :] + float(b["sigma"][s]) * z).reshape(-1))
    return torch.cat(parts).contiguous()


def surrogate_leg(a, ctx, opmm, torch, synth, keep=False):
    """Learned seed vs plain search on held-out saccades of the same distributions: the network is
    trained on the device on saccades the plant simulator generates (OPC = nominal x U[0.7, 1.3],
    noise sigma U[0, 0.1] deg), then seeds a small refine; saccades whose seeded RMSE exceeds
    1.5 sigma fall back to the plain search, which also fits every held-out saccade for reference."""
    B = 4096
    steps = max(1, a.train_saccades // B)
    sg = opmm.Surrogate(ctx, init_seed=20070988)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = sg.train(data_seed=1, batch=B, n_steps=steps, lr0=2e-3, lr_min=2e-5)
    train_s = time.perf_counter() - t0
    # the training kernels' share of the BF16 MFMA peak: forward + backward of one generated batch (one fused
    # kernel for the forward pass, the loss and the input gradients, one for the four layers' weight
    # gradients; the loss is not returned, so not reset), timed with HIP events
    feat = torch.empty(B, 256, dtype=torch.int16, device="cuda")
    target = torch.empty(B, 18, dtype=torch.float32, device="cuda")
    sg.generate(1, 0, feat, target)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        sg.backward(feat, target, want_loss=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record(stream)
    for _ in range(reps):
        sg.backward(feat, target, want_loss=False)
    e1.record(stream)
    torch.cuda.synchronize()
    fb_ms = e0.elapsed_time(e1) / reps
    fb_flop = 2.0 * B * (2 * MLP_MACS + MLP_DX_MACS)
    fb = {"batch": B, "ms": fb_ms, "flop": fb_flop, "tflops": fb_flop / (fb_ms * 1e-3) / 1e12,
          "mfma_frac": fb_flop / (fb_ms * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS}
    b = synth.draw_saccades(a.heldout, "full", seed=synth.BASE_SEED + 1)
    pos = gpu_targets(ctx, opmm, torch, b)
    recs = opmm.saccade_records(b["T"], 2, b["amp"], b["dir_deg"], b["dur_ms"], b["seed"])
    S = a.heldout
    # both searches screen their rounds like the main fit (same results as FP64 only)
    scr_plain, scr_seed = min(a.screen_rounds, a.rounds), min(a.screen_rounds, a.seed_rounds)
    plain = opmm.fit_params(n_cand=a.n_cand, n_rounds=a.rounds, mode=opmm.FIT_ROUNDS, screen_rounds=scr_plain,
                            screen_tol=a.screen_tol)
    seeded = opmm.fit_params(n_cand=a.seed_cand, n_rounds=a.seed_rounds, w_init_frac=a.seed_width,
                             mode=opmm.FIT_ROUNDS, screen_rounds=scr_seed, screen_tol=a.screen_tol)
    opc = torch.zeros(S, 18, device="cuda")
    rm_plain = torch.zeros(S, device="cuda")
    rm_seed = torch.zeros(S, device="cuda")
    st = torch.zeros(S, dtype=torch.int32, device="cuda")
    ctx.fit(pos, recs, plain, opc, rm_plain)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.fit(pos, recs, plain, opc, rm_plain)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    sg.fit(pos, recs, seeded, plain, 1.5 * synth.SIGMA, opc, rm_seed, st)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_fb = sg.fit(pos, recs, seeded, plain, 1.5 * synth.SIGMA, opc, rm_seed, st)
    torch.cuda.synchronize()
    seed_s = time.perf_counter() - t0
    rp, rs = rm_plain.cpu().numpy(), rm_seed.cpu().numpy()
    # gradient polish (exact sensitivities + Levenberg-Marquardt) after the seeded refine, and after the
    # plain search for reference
    pprm = opmm.polish_params(max_iter=a.polish_iter)
    opc_p = opc.clone()
    rm_sp = torch.zeros(S, device="cuda")
    its = torch.zeros(S, dtype=torch.int32, device="cuda")
    ctx.polish(pos, recs, pprm, opc_p, rm_sp, iters_out=its)  # warm-up
    opc_p.copy_(opc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.polish(pos, recs, pprm, opc_p, rm_sp, iters_out=its)
    torch.cuda.synchronize()
    pol_s = time.perf_counter() - t0
    rsp, itn = rm_sp.cpu().numpy(), its.cpu().numpy()
    opc_pp = torch.zeros(S, 18, device="cuda")
    ctx.fit(pos, recs, plain, opc_pp, rm_plain)
    rm_pp = torch.zeros(S, device="cuda")
    ctx.polish(pos, recs, pprm, opc_pp, rm_pp)
    rpp = rm_pp.cpu().numpy()
    if not keep:
        sg.close()
        sg = None
    return sg, {"train": {"saccades": steps * B, "steps": steps, "batch": B, "seconds": train_s,
                      "loss_first": float(loss[:10].mean()), "loss_last": float(loss[-10:].mean()),
                      "step_ms": 1e3 * train_s / steps, "forward_backward": fb},
            "heldout_saccades": S,
            "plain": {"n_cand": a.n_cand, "rounds": a.rounds, "screen_rounds": scr_plain,
                      "saccades_fitted_per_s": S / plain_s,
                      "mean_rmse_deg": float(rp.mean()), "median_rmse_deg": float(np.median(rp))},
            "surrogate": {"n_cand": a.seed_cand, "rounds": a.seed_rounds, "screen_rounds": scr_seed,
                          "w_init_frac": a.seed_width,
                          "fallback_rmse_deg": 1.5 * synth.SIGMA, "fallbacks": int(n_fb),
                          "saccades_fitted_per_s": S / seed_s, "mean_rmse_deg": float(rs.mean()),
                          "median_rmse_deg": float(np.median(rs))},
            "surrogate_polished": {"polish_max_iter": a.polish_iter, "mean_polish_iters": float(itn.mean()),
                                   "saccades_fitted_per_s": S / (seed_s + pol_s),
                                   "polish_seconds": pol_s, "mean_rmse_deg": float(rsp.mean()),
                                   "median_rmse_deg": float(np.median(rsp)),
                                   "not_worse_than_plain": float(np.mean(rsp <= rp * (1 + 1e-6)))},
            "plain_polished": {"mean_rmse_deg": float(rpp.mean()), "median_rmse_deg": float(np.median(rpp))},
            "speedup_saccades_per_s": plain_s / (seed_s + pol_s),
            "rmse_ratio_surrogate_over_plain": float(rsp.mean() / rp.mean()),
            "refine_only": {"speedup_saccades_per_s": plain_s / seed_s,
                            "rmse_ratio_surrogate_over_plain": float(rs.mean() / rp.mean())}}


def uneven_leg(a, ctx, opmm, torch, synth):
    """Batched uneven saccades: 4096 saccades of 20-150 samples, per-saccade candidate counts from
    {4096, 16384, 65536}, every round of every saccade in one persistent launch captured in a graph,
    shape picked by the autotuner; the per-round launches of the default shape beside it."""
    b = synth.draw_saccades(4096, "uneven", seed=synth.BASE_SEED + 2)
    pos = gpu_targets(ctx, opmm, torch, b)
    recs = opmm.saccade_records(b["T"], 2, b["amp"], b["dir_deg"], b["dur_ms"], b["seed"], n_cand=b["n_cand"])
    S, R = 4096, a.rounds
    sims = int(np.sum(b["n_cand"].astype(np.int64))) * R
    opc = torch.zeros(S, 18, device="cuda")
    rm = torch.zeros(S, device="cuda")
    out = {"saccades": S, "rounds": R, "candidate_sims_per_step": sims, "mean_T": float(np.mean(b["T"]))}
    variants = [("persistent", opmm.FIT_PERSISTENT, 0), ("rounds", opmm.FIT_ROUNDS, 0)]
    if a.screen_rounds > 0:
        variants.append(("rounds_screened", opmm.FIT_ROUNDS, min(a.screen_rounds, R)))
    fitted = {}
    for name, mode, scr in variants:
        p = opmm.fit_params(n_cand=4096, n_rounds=R, mode=mode)
        p.tile = ctx.autotune(pos, recs, p) if name == "persistent" else opmm.lib.opmm_tile_default()
        if scr:
            p.screen_rounds, p.screen_tol = scr, a.screen_tol
        pl = ctx.plan(pos, recs, p, opc, rm)
        pl.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            pl.launch()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 3
        pl.close()
        out[name] = {"tile": opmm.tile_names()[p.tile], "ms_per_step": dt * 1e3, "candidate_sims_per_s": sims / dt,
                     "saccades_fitted_per_s": S / dt}
        fitted[name] = opc.clone()
        if scr:
            out[name].update(screen_rounds=scr, same_opc_as_fp64=bool(torch.equal(fitted[name], fitted["rounds"])))
    return out


def tiny_leg(a, ctx, opmm, torch, synth):
    """The tiny configuration: one horizontal 10 deg saccade (T = 80, one channel), 4096 candidates,
    one argmin pass; latency of one captured fit, launch to synchronise."""
    b = synth.draw_saccades(1, "tiny")
    pos = gpu_targets(ctx, opmm, torch, b)
    recs = opmm.saccade_records(b["T"], 1, b["amp"], b["dir_deg"], b["dur_ms"], b["seed"])
    opc = torch.zeros(1, 18, device="cuda")
    rm = torch.zeros(1, device="cuda")
    pl = ctx.plan(pos, recs, opmm.fit_params(n_cand=4096, n_rounds=1), opc, rm)
    for _ in range(5):
        pl.launch()
    torch.cuda.synchronize()
    lat = []
    for _ in range(100):
        t0 = time.perf_counter()
        pl.launch()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    pl.close()
    return {"n_cand": 4096, "rounds": 1, "latency_ms_p50": float(np.percentile(lat, 50)),
            "latency_ms_p99": float(np.percentile(lat, 99)), "rmse_deg": float(rm.item())}


def ivt_leg(a, ctx, opmm, torch, synth):
    """I-VT on a synthetic 1 kHz gaze stream: fixations of 100-300 ms (0.003 deg noise) joined by
    plant-simulated saccades with the full configuration's amplitude, direction and duration draws
    (true OPC = nominal x U[0.8, 1.2]).  Timed: one extraction call, records back on the host."""
    rng = np.random.default_rng(synth.BASE_SEED + 5)
    n = a.ivt_saccades
    amp = rng.uniform(2.0, 30.0, n)
    phi = np.radians(rng.uniform(0.0, 360.0, n))
    dur = 2.2 * amp + 21.0
    T = np.ceil(dur).astype(np.int64) + 30           # the saccade and its settling
    fix = rng.integers(100, 301, n)
    true = np.stack([opmm.nominal(float(d)) for d in dur]) * rng.uniform(0.8, 1.2, (n, 18)).astype(np.float32)
    Tmax = int(T.max())
    theta = torch.zeros(n, Tmax, device="cuda")
    ctx.simulate(torch.from_numpy(true.astype(np.float32)).cuda(), torch.from_numpy(amp.astype(np.float32)).cuda(),
                 Tmax, theta)
    th = theta.cpu().numpy()
    parts, p = [], np.zeros(2)
    for i in range(n):
        u = np.array([math.cos(phi[i]), math.sin(phi[i])])
        parts.append(np.tile(p, (int(fix[i]), 1)))
        parts.append(p + th[i, :T[i], None] * u[None, :])
        p = p + amp[i] * u
    parts.append(np.tile(p, (200, 1)))
    g = np.concatenate(parts)
    g = (g + 0.003 * rng.standard_normal(g.shape)).astype(np.float32)
    gaze = torch.from_numpy(g).cuda()
    pos_out = torch.empty(2 * g.shape[0], device="cuda")
    ctx.ivt_extract(gaze, pos_out, max_out=n + 64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs, src = ctx.ivt_extract(gaze, pos_out, max_out=n + 64)
    ivt_s = time.perf_counter() - t0
    out = {"stream_samples": int(g.shape[0]), "stream_seconds": g.shape[0] * 1e-3, "planted": n,
           "extracted": int(len(recs)), "seconds": ivt_s, "samples_per_s": g.shape[0] / ivt_s,
           "realtime_factor": g.shape[0] * 1e-3 / ivt_s}
    return out


def nm_leg(a, ctx, opmm, torch, pos, recs, rm_box, box_s):
    """The paper's estimator (parallel Nelder-Mead, one task per saccade, all transforms of an
    iteration at once) on the same batch, from the nominal OPC, against the box search."""
    S = recs.shape[0]
    prm = opmm.nm_params(max_iter=a.nm_iter, tol_x=1e-4, tol_f=1e-6)
    opc = torch.zeros(S, 18, device="cuda")
    rm = torch.zeros(S, device="cuda")
    it = torch.zeros(S, dtype=torch.int32, device="cuda")
    ctx.fit_nm(pos, recs, prm, opc, rm, it)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.fit_nm(pos, recs, prm, opc, rm, it)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r, its = rm.cpu().numpy(), it.cpu().numpy()
    out = {"max_iter": a.nm_iter, "tol_x": 1e-4, "tol_f": 1e-6, "saccades_fitted_per_s": S / dt,
           "mean_rmse_deg": float(r.mean()), "mean_iters": float(its.mean()),
           "converged": int(np.count_nonzero(its < a.nm_iter)),
           "box_search_saccades_fitted_per_s": S / box_s, "box_search_mean_rmse_deg": float(rm_box.mean())}
    # a batch that oversubscribes the device's waves: 4096 saccades of the same distributions, one or
    # two tasks per wave (auto picks two here)
    from paper_2007_09884_amd import synth
    b = synth.draw_saccades(4096, "full", seed=synth.BASE_SEED + 4)
    pos4 = gpu_targets(ctx, opmm, torch, b)
    recs4 = opmm.saccade_records(b["T"], 2, b["amp"], b["dir_deg"], b["dur_ms"], b["seed"])
    S4 = 4096
    opc4 = torch.zeros(S4, 18, device="cuda")
    rm4 = torch.zeros(S4, device="cuda")
    big = {}
    for name, g in (("one_per_wave", 1), ("two_per_wave", 2)):
        prm4 = opmm.nm_params(max_iter=a.nm_iter, tol_x=1e-4, tol_f=1e-6, tasks_per_wave=g)
        ctx.fit_nm(pos4, recs4, prm4, opc4, rm4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.fit_nm(pos4, recs4, prm4, opc4, rm4)
        torch.cuda.synchronize()
        big[name] = S4 / (time.perf_counter() - t0)
    big["mean_rmse_deg"] = float(rm4.cpu().numpy().mean())
    out["saccades_4096"] = big
    return out


def note(msg):
    """Progress of the legs on stderr (the JSON line on stdout stays the only output there)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def serve_leg(a, ctx, opmm, torch, synth, sg, rates=None, polish_iter=0, seconds=None, pool=50000):
    """Continuous batching: saccades of the full-estimation distributions arrive as a Poisson stream;
    the server admits them into device slots, seeds them from the learned network, advances every
    resident request by one round per step (and, with polish_iter, polishes each finished search).
    Latency = arrival to result on the host.  Requests beyond `pool` distinct synthetic saccades reuse
    their traces with seeds of their own (so each still runs its own candidate stream)."""
    rates = rates or [float(r) for r in a.serve_rates.split(",") if r]
    seconds = a.serve_seconds if seconds is None else seconds
    out = []
    for lam in rates:
        n = max(16, int(lam * seconds))
        m = min(n, pool)
        b = synth.draw_saccades(m, "full", seed=synth.BASE_SEED + 100 + int(lam))
        pos = gpu_targets(ctx, opmm, torch, b).cpu().numpy()
        base = opmm.saccade_records(b["T"], 2, b["amp"], b["dir_deg"], b["dur_ms"], b["seed"])
        recs = base[np.arange(n) % m]
        if n > m:
            recs["seed"] = (np.uint64(synth.BASE_SEED) * np.uint64(1000003) + np.arange(n, dtype=np.uint64))
        rng = np.random.default_rng(int(lam))
        arrive = np.cumsum(rng.exponential(1.0 / lam, n))
        prm = opmm.serve_params(max_slots=65536, hbm_budget_bytes=1 << 30, fallback_rmse=1.5 * synth.SIGMA,
                                polish_iter=polish_iter)
        prm.seeded.n_cand, prm.seeded.n_rounds, prm.seeded.w_init_frac = a.seed_cand, a.seed_rounds, a.seed_width
        prm.plain.n_cand, prm.plain.n_rounds = 16384, 10
        sv = opmm.Server(ctx, prm, sg)
        gc.collect()
        gc.disable()  # a collector pass inside the arrival loop would show up as request latency
        t0 = sv.now()
        nxt, done, lat, rm, fb = 0, 0, [], [], 0
        while done < n:
            now = sv.now() - t0
            k = int(np.searchsorted(arrive, now, side="right"))
            if k > nxt:
                sv.submit_many(pos, recs[nxt:k], t0 + arrive[nxt:k])
                nxt = k
            sv.step()
            r = sv.poll()
            done += len(r["id"])
            lat.append(r["t_done"] - r["t_arrival"])
            rm.append(r["rmse"])
            fb += int(np.count_nonzero(r["status"] & opmm.ST_FALLBACK))
        span = sv.now() - t0
        gc.enable()
        st = sv.stats()
        sv.close()
        lat = np.concatenate(lat) * 1e3
        out.append({"rate_per_s": lam, "window_s": seconds, "requests": n, "distinct_traces": m,
                    "p50_ms": float(np.percentile(lat, 50)),
                    "p99_ms": float(np.percentile(lat, 99)), "p999_ms": float(np.percentile(lat, 99.9)),
                    "sustained_per_s": n / span,
                    "mean_rmse_deg": float(np.concatenate(rm).mean()), "fallbacks": fb, "steps": st["steps"],
                    "slots": st["slots"], "polish_iter": polish_iter})
    return out


def cpu_baseline(b, pos_host, seconds):
    """The FP64 oracle's own box search (candidate draw + RK4 simulation + RMSE + argmin), one round,
    on a bounded sample of the same workload, all host cores."""
    import oracle
    cores = min(16, len(os.sched_getaffinity(0)))  # the host share of one GPU
    s = 0
    T = int(b["T"][s])
    amp, phi, dur = (float(np.float32(b[k][s])) for k in ("amp", "dir_deg", "dur_ms"))
    probe = 2000
    t0 = time.perf_counter()
    oracle.fit(pos_host[0], amp, phi, dur, int(b["seed"][s]), probe, 1, nthreads=cores)
    rate = probe / (time.perf_counter() - t0)
    n = int(max(probe, min(rate * seconds, 8_000_000)))
    t0 = time.perf_counter()
    oracle.fit(pos_host[0], amp, phi, dur, int(b["seed"][s]), n, 1, nthreads=cores)
    dt = time.perf_counter() - t0
    # the same search on one thread, as the paper's serial implementation ran (a ~2 s sample)
    n1 = int(max(200, min(rate / cores * 2.0, 1_000_000)))
    t0 = time.perf_counter()
    oracle.fit(pos_host[0], amp, phi, dur, int(b["seed"][s]), n1, 1, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": n / dt, "unit": "candidate-sims/s", "cores": cores, "kind": "oracle",
            "sample": "saccade 0 of the batch (T=%d, 2 channels), one round of %d candidates: FP64 RK4 "
                      "(16 substeps/ms) + RMSE + argmin, %.1f s on %d threads" % (T, n, dt, cores),
            "single_thread": {"value": n1 / dt1, "candidates": n1, "seconds": dt1}}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the estimation shards by saccade with no exchange, and this "
              "build measures the one-GPU share; --gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    if a.copy_probe:
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel(), "launches": 3}))
        return

    from paper_2007_09884_amd import opmm, synth

    torch.cuda.init()
    b = synth.draw_saccades(a.saccades, "full")
    ctx = opmm.Context(0)
    pos = gpu_targets(ctx, opmm, torch, b)
    recs = opmm.saccade_records(b["T"], 2, b["amp"], b["dir_deg"], b["dur_ms"], b["seed"])
    S, N, R = a.saccades, a.n_cand, a.rounds
    opc = torch.zeros(S, 18, device="cuda")
    rmse = torch.zeros(S, device="cuda")
    status = torch.zeros(S, dtype=torch.int32, device="cuda")
    modes = {"persistent": opmm.FIT_PERSISTENT, "rounds": opmm.FIT_ROUNDS}

    def time_plan(p, reps=2):
        """ms of one captured step with fit parameters p, after a warm-up launch"""
        pl = ctx.plan(pos, recs, p, opc, rmse, None, status)
        pl.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pl.launch()
        torch.cuda.synchronize()
        pl.close()
        return (time.perf_counter() - t0) / reps * 1e3

    def autotuned(name):
        p = opmm.fit_params(n_cand=N, n_rounds=R, mode=modes[name])
        p.tile = ctx.autotune(pos, recs, p)
        return p

    tuned = {}
    if a.mode == "auto" or not a.no_autotune_leg:
        # the project's autotuner on both launch modes, each pick timed on a whole step
        for name in ("persistent", "rounds"):
            p = autotuned(name)
            tuned[name] = {"tile": opmm.tile_names()[p.tile], "ms_per_step": time_plan(p), "params": p}
    if a.mode == "auto":
        a.mode = min(tuned, key=lambda k: tuned[k]["ms_per_step"])
        prm = tuned[a.mode]["params"]
    else:
        prm = opmm.fit_params(n_cand=N, n_rounds=R, mode=modes[a.mode])
        prm.tile = autotuned(a.mode).tile if a.tile == -2 else a.tile
    if prm.tile < 0:
        prm.tile = opmm.lib.opmm_tile_default()
    if a.screen_rounds > 0 and prm.mode == opmm.FIT_ROUNDS:
        prm.screen_rounds, prm.screen_tol = min(a.screen_rounds, R), a.screen_tol
    for v in tuned.values():
        del v["params"]
    torch.cuda.synchronize()

    if a.no_graph:
        def step():
            ctx.fit(pos, recs, prm, opc, rmse, None, status)
    else:
        plan = ctx.plan(pos, recs, prm, opc, rmse, None, status)

        def step():
            plan.launch()

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms_gpu = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))  # captured step, launch stream

    sims = S * N * R
    ms_per_step = wall / a.steps * 1e3
    value = sims * a.steps / wall
    sum_T = int(np.sum(b["T"]))
    flop = FLOP_PER_CAND_SAMPLE * N * R * sum_T
    scr = int(prm.screen_rounds)
    tile_name = opmm.tile_names()[prm.tile]
    # Each search kernel's own launches, timed by the library's event pairs on the launch stream over
    # `steps` more fits of the same batch queued directly (a captured plan cannot be split by kernel).
    ctx.kernel_timing(True)
    for _ in range(a.steps):
        ctx.fit(pos, recs, prm, opc, rmse, None, status)
    kt = {}
    for kid, kname in ((opmm.KERNEL_ROUND, "fit_round_kernel"), (opmm.KERNEL_SCREEN, "fit_screen_kernel"),
                       (opmm.KERNEL_VERIFY, "fit_verify_kernel"), (opmm.KERNEL_PERSISTENT, "fit_persistent_kernel")):
        tot, n = ctx.kernel_times(kid)
        if n:
            kt[kname] = {"avg_ms": tot / n, "launches_per_step": n / a.steps, "ms_per_step": tot / a.steps}
    ctx.kernel_timing(False)
    dom = max(kt, key=lambda k: kt[k]["ms_per_step"])
    # the algorithmic unit: one recurrence step of one candidate (54 FLOP); a round kernel or a screen
    # kernel covers one round of the batch, the persistent kernel the whole step
    flop_launch = flop if dom == "fit_persistent_kernel" else flop // R
    fp32 = dom == "fit_screen_kernel"
    peak = PUBLISHED_FP32_PEAK if fp32 else ALU_PEAK_TFLOPS
    dom_ms = kt[dom]["avg_ms"]
    achieved = flop_launch / (dom_ms * 1e-3) / 1e12
    # the whole step against the peak of the precision each round runs in
    step_peak = R / (scr / PUBLISHED_FP32_PEAK + (R - scr) / ALU_PEAK_TFLOPS)
    step_tflops = flop / (step_ms_gpu * 1e-3) / 1e12
    if scr > 0:
        kernel_text = ("fit_screen_kernel: the FP32 pass over every candidate of one screened round "
                       "(%d of %d rounds are screened; their survivors within %.0e deg RMSE of the FP32 best go "
                       "to fit_verify_kernel in FP64; the other rounds run fit_round_kernel in FP64)" % (
                           scr, R, prm.screen_tol))
    elif dom == "fit_persistent_kernel":
        kernel_text = "fit_persistent_kernel: one work-queue launch for the whole step, FP64 recurrence"
    else:
        kernel_text = "fit_round_kernel: every candidate of one round, FP64 recurrence (%d launches per step)" % R
    st = status.cpu().numpy()
    rm = rmse.cpu().numpy()

    out = {
        "metric": "OPC candidate sims/s; saccades fitted/s at equal RMSE, surrogate vs plain",
        "value": value,
        "unit": "candidate-sims/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 screen + f64 verify" if scr > 0 else "f64",
        "data": "synthetic",
        "config": {"workload": "full estimation: %d 2-D saccades (A~U[2,30] deg, D=2.2A+21 ms, 1 kHz), "
                               "%d candidates x %d halving rounds, plain box search" % (S, N, R),
                   "saccades": S, "n_cand": N, "rounds": R, "mean_T": float(np.mean(b["T"])),
                   "mode": a.mode, "graph": not a.no_graph, "tile": opmm.tile_names()[prm.tile],
                   "screen_rounds": int(prm.screen_rounds), "screen_tol_deg": float(prm.screen_tol)},
        "saccades_fitted_per_s": S * a.steps / wall,
        "mean_final_rmse_deg": float(np.mean(rm)),
        "status_nonzero": int(np.count_nonzero(st)),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": profiled_value("traffic_per_launch_bytes", dom, tile_name),
                     "kernel": kernel_text,
                     "peak_source": ("published FP32 vector peak (non-packed FMA issues at up to twice the FP64 "
                                     "rate on this chip)" if fp32 else
                                     "FP64 vector peak: 256 CU x 4 SIMD x 16 lanes x FMA x 2.4 GHz"),
                     "launch_ms": dom_ms, "launch_timing": "library event pairs around each launch, launch stream",
                     "algorithmic_flop_per_launch": flop_launch,
                     "executed": executed_fig(profiled_value("executed_flop_per_launch", dom, tile_name), dom_ms,
                                              peak),
                     "kernels": kt,
                     "step": {"achieved": step_tflops, "peak": step_peak, "frac": step_tflops / step_peak,
                              "note": "whole captured step (all kernels) against the peak of each round's "
                                      "precision: %d FP32 rounds at %.1f, %d FP64 rounds at %.1f TFLOP/s" % (
                                          scr, PUBLISHED_FP32_PEAK, R - scr, ALU_PEAK_TFLOPS)}},
    }
    if a.report_csv:
        # one more fit (untimed) for the mean absolute difference, the paper's OptErr; the serial
        # re-check column (CPU_check) is left empty here
        from paper_2007_09884_amd import report
        mae = torch.zeros(S, device="cuda")
        ctx.fit(pos, recs, prm, opc, rmse, mae, status)
        report.write_csv(a.report_csv, opc.cpu().numpy(), mae.cpu().numpy())
    if scr > 0 and not a.no_fp64_leg:
        # the same workload with every round in FP64 only: its time, and that it returns the same fit
        p64 = opmm.fit_params(n_cand=N, n_rounds=R, mode=modes[a.mode], tile=prm.tile)
        opc_s = opc.clone()
        ms64 = time_plan(p64, reps=5)
        out["fp64_only"] = {"ms_per_step": ms64, "candidate_sims_per_s": sims / (ms64 * 1e-3),
                            "step_frac_of_fp64_peak": flop / (ms64 * 1e-3) / 1e12 / ALU_PEAK_TFLOPS,
                            "same_opc_as_screened": bool(torch.equal(opc, opc_s))}
    if tuned:
        out["autotune"] = tuned
    if not a.no_uneven:
        note("batched uneven")
        out["batched_uneven"] = uneven_leg(a, ctx, opmm, torch, synth)
    if not a.no_model9:
        # the 9-parameter model (Table 2) on the same batch and launch
        p9 = opmm.fit_params(n_cand=N, n_rounds=R, mode=modes[a.mode], tile=prm.tile, model=9,
                             screen_rounds=scr, screen_tol=prm.screen_tol)
        ms9 = time_plan(p9, reps=3)
        out["model9"] = {"ms_per_step": ms9, "candidate_sims_per_s": sims / (ms9 * 1e-3), "screen_rounds": scr,
                         "mean_final_rmse_deg": float(rmse.mean().item())}
    if not a.no_ivt:
        note("I-VT")
        out["ivt"] = ivt_leg(a, ctx, opmm, torch, synth)
    if not a.no_tiny:
        note("tiny configuration")
        out["tiny"] = tiny_leg(a, ctx, opmm, torch, synth)
    if not a.no_nm:
        note("Nelder-Mead")
        out["nelder_mead"] = nm_leg(a, ctx, opmm, torch, pos, recs, rm, ms_per_step * 1e-3)
    if not a.no_surrogate:
        note("learned seed")
        sg, out["surrogate_vs_plain"] = surrogate_leg(a, ctx, opmm, torch, synth, keep=not a.no_serve)
        if not a.no_serve:
            note("serving")
            out["serving"] = serve_leg(a, ctx, opmm, torch, synth, sg)
            if a.serve_long_seconds > 0:
                note("serving, %.0f s window at %.0f/s" % (a.serve_long_seconds, a.serve_long_rate))
                out["serving_long"] = serve_leg(a, ctx, opmm, torch, synth, sg, rates=[a.serve_long_rate],
                                                seconds=a.serve_long_seconds)[0]
            if a.serve_polish > 0:
                out["serving_polished"] = serve_leg(a, ctx, opmm, torch, synth, sg, rates=[20000.0],
                                                    polish_iter=a.serve_polish)
            sg.close()
    if not a.no_cpu_baseline:
        pos_host = []
        off = 0
        ph = pos.cpu().numpy()
        for s in range(1):
            T = int(b["T"][s])
            pos_host.append(ph[off:off + 2 * T].reshape(T, 2))
        note("oracle on the host")
        out["cpu_baseline"] = cpu_baseline(b, pos_host, a.cpu_seconds)
    out["paper_figures"] = PAPER_FIGURES
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
