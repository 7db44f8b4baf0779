"""Pins for the FP64 oracle: checks against things other than itself.

Each test states what fixes the expected value: a number the paper prints, a
published test vector, a library routine (scipy's matrix exponential), a
closed form derived by hand from the model reading, an invariance of the
equations, or brute force on a tiny grid.  A plausible slip in the oracle
(dropped term, wrong sign, swapped muscle, wrong unit) fails at least one.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2007_09884_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FORCE_TYPE = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 14, 15, 16]  # K_SE, K_LT, B, B_P, N_C, J, N_C_FIX, N_SAC


def rand_opc(rng, dur=43.0, lo=0.7, hi=1.3):
    return oracle.nominal(dur) * rng.uniform(lo, hi, 18)


# --- values the paper prints / published vectors ---------------------------------------------

def test_table1_nominal_matches_paper():
    """Section 2.2.1, Table 1: nominal values and order; PW = duration - 6 ms."""
    rows = [l.split() for l in open(os.path.join(GOLD, "table1_nominal.txt")) if not l.startswith("#")]
    nom = oracle.nominal(43.0)
    for j, (name, val) in enumerate(rows[:17]):
        assert nom[j] == float(val), name
    assert rows[17] == ["PW", "duration-6"] and nom[17] == 37.0
    assert oracle.nominal(100.0)[17] == 94.0


def test_splitmix64_published_vectors():
    lines = [l.split() for l in open(os.path.join(GOLD, "splitmix64_vectors.txt")) if not l.startswith("#")]
    seed = int(lines[0][1])
    for n, row in enumerate(lines[1:], start=1):
        assert oracle.splitmix64(seed, n) == int(row[0])


# --- integrator vs the matrix-exponential closed form ----------------------------------------

def _affine_system(p, n_ag, n_ant, tau_ag, tau_ant):
    """x' = A x + b read off the oracle's right-hand side by probing (the plant is affine)."""
    b = oracle.rhs(p, np.zeros(6), n_ag, n_ant, tau_ag, tau_ant)
    A = np.zeros((6, 6))
    for j in range(6):
        e = np.zeros(6); e[j] = 1.0
        A[:, j] = oracle.rhs(p, e, n_ag, n_ant, tau_ag, tau_ant) - b
    # affine check: rhs of a random point is A x + b
    x = np.random.default_rng(0).normal(size=6)
    assert np.allclose(oracle.rhs(p, x, n_ag, n_ant, tau_ag, tau_ant), A @ x + b, rtol=1e-12, atol=1e-9)
    return A, b


def _expm_flow(A, b, x, t):
    """Exact solution after time t of x' = A x + b, via the augmented exponential."""
    M = np.zeros((7, 7)); M[:6, :6] = A; M[:6, 6] = b
    return (scipy.linalg.expm(M * t) @ np.append(x, 1.0))[:6]


@pytest.mark.parametrize("case", range(6))
def test_rk4_matches_matrix_exponential(case):
    """Piecewise-LTI closed form x(t) = e^{A_k (t-t_k)} applied piecewise, at every sample,
    including the sample split at PW (non-integer PW)."""
    rng = np.random.default_rng(100 + case)
    amp = rng.uniform(2, 30)
    dur = 2.2 * amp + 21
    p = rand_opc(rng, dur)
    T = int(math.ceil(dur)) + 20
    lv = oracle.control_levels(p, amp)
    th, st = oracle.simulate_levels(p, lv, T, states=True)
    th32 = oracle.simulate_levels(p, lv, T, nsub=32)
    A1, b1 = _affine_system(p, lv[2], lv[3], p[10] * 1e-3, p[11] * 1e-3)
    A2, b2 = _affine_system(p, lv[4], lv[5], p[12] * 1e-3, p[13] * 1e-3)
    x0 = st[0]
    pw = p[17] * 1e-3
    xpw = _expm_flow(A1, b1, x0, pw)
    ref = []
    for k in range(T):
        t = k * 1e-3
        x = _expm_flow(A1, b1, x0, t) if t <= pw else _expm_flow(A2, b2, xpw, t - pw)
        ref.append(x[0])
    err = np.abs(th - np.array(ref)).max()
    err32 = np.abs(th32 - np.array(ref)).max()
    assert err < 3e-9, err                  # the oracle's default: 16 RK4 substeps per sample
    assert err32 < err / 10 or err32 < 1e-11  # fourth-order convergence towards the closed form
    # the sample grid really straddles PW
    assert 0 < pw * 1e3 < T - 1 and pw * 1e3 != int(pw * 1e3)


# --- invariants and hand-derived closed forms -------------------------------------------------

def test_initial_state_is_equilibrium_and_theta0_zero():
    rng = np.random.default_rng(1)
    for _ in range(20):
        p = rand_opc(rng)
        lv = oracle.control_levels(p, rng.uniform(2, 30))
        x0 = oracle.equilibrium(p, lv[0], lv[1])
        dx = oracle.rhs(p, x0, lv[0], lv[1], 1e-3, 1e-3)
        assert np.abs(dx).max() < 1e-9 * max(1.0, np.abs(x0).max() / p[9])
        assert abs(x0[0]) < 1e-13
        # any constant active state: the closed-form statics zero every derivative
        fa, fn = rng.uniform(0, 80), rng.uniform(0, 40)
        xe = oracle.equilibrium(p, fa, fn)
        de = oracle.rhs(p, xe, fa, fn, 1e-3, 1e-3)
        assert abs(xe[0]) > 1e-3
        assert np.abs(de).max() < 1e-9 * max(1.0, np.abs(xe).max() / p[9])


def test_zero_deviation_input_gives_no_motion():
    rng = np.random.default_rng(2)
    p = rand_opc(rng)
    lv = oracle.control_levels(p, 10.0)
    flat = np.array([lv[0], lv[1]] * 3)
    th = oracle.simulate_levels(p, flat, 120)
    assert np.abs(th).max() < 1e-12


def test_negated_control_and_superposition():
    """With the same time-constant schedule the plant is linear in the deviation of the
    control from the resting levels: negation and superposition hold."""
    rng = np.random.default_rng(3)
    p = rand_opc(rng)
    base = oracle.control_levels(p, 0.0)
    s0 = np.array([base[0], base[1]] * 3)
    d1 = np.array([0, 0, 30.0, -10.0, 5.0, -3.0])
    d2 = np.array([0, 0, -7.0, 4.0, -2.0, 6.0])
    t1 = oracle.simulate_levels(p, s0 + d1, 100)
    tneg = oracle.simulate_levels(p, s0 - d1, 100)
    t2 = oracle.simulate_levels(p, s0 + d2, 100)
    t12 = oracle.simulate_levels(p, s0 + d1 + d2, 100)
    scale = np.abs(t1).max()
    assert np.abs(t1 + tneg).max() < 1e-11 * scale
    assert np.abs(t12 - (t1 + t2)).max() < 1e-11 * scale


def test_steady_state_equals_amplitude():
    """The post-saccadic step holds the eye at the amplitude (fixation statics)."""
    rng = np.random.default_rng(4)
    for _ in range(6):
        amp = rng.uniform(2, 30)
        p = rand_opc(rng, 2.2 * amp + 21)
        th = oracle.simulate(p, amp, 3000, nsub=4)
        assert abs(th[-1] - amp) < 1e-8, (th[-1], amp)


def test_steady_state_arbitrary_levels_force_balance():
    """Statics derived by hand: c_m = K_SE/(K_SE+K_LT); the globe balances
    c_AG(F_AG - K_LT_AG th) - c_ANT(F_ANT + K_LT_ANT th) = K_P th with K_P = N_C_AG + N_C_ANT."""
    rng = np.random.default_rng(5)
    p = rand_opc(rng)
    lv = np.array([0.0, 0.0, 40.0, 3.0, 31.0, 12.0])
    lv[0], lv[1] = oracle.control_levels(p, 0.0)[:2]
    th = oracle.simulate_levels(p, lv, 3000, nsub=4)
    ca = p[0] / (p[0] + p[2]); cn = p[1] / (p[1] + p[3])
    kp = p[7] + p[8]
    ss = (ca * lv[4] - cn * lv[5]) / (kp + ca * p[2] + cn * p[3])
    assert abs(th[-1] - ss) < 1e-8


def test_force_scale_gauge():
    """Scaling every force-type parameter (13 of them) by k leaves theta(t) unchanged."""
    rng = np.random.default_rng(6)
    p = rand_opc(rng)
    q = p.copy(); q[FORCE_TYPE] *= 3.7
    a = oracle.simulate(p, 12.0, 90); b = oracle.simulate(q, 12.0, 90)
    assert np.abs(a - b).max() < 1e-11 * np.abs(a).max()
    # and a non-gauge change (one parameter only) does change it
    q2 = p.copy(); q2[9] *= 3.7
    assert np.abs(oracle.simulate(q2, 12.0, 90) - a).max() > 1e-3


def test_time_scale_invariance():
    """t -> k t: time constants and PW scale by k, viscosities by k, inertia by k^2;
    sampled every k ms the trajectory is the same."""
    rng = np.random.default_rng(7)
    p = rand_opc(rng)
    k = 2.0
    q = p.copy()
    q[[10, 11, 12, 13, 17]] *= k
    q[[4, 5, 6]] *= k
    q[9] *= k * k
    a = oracle.simulate(p, 15.0, 80, dt_ms=1.0)
    b = oracle.simulate(q, 15.0, 80, dt_ms=k)
    assert np.abs(a - b).max() < 1e-11 * np.abs(a).max()


def test_onset_fourth_derivative():
    """Right after pulse onset, from rest: F_m jumps in slope (N_SAC_m - S_m(0))/tau_AC_m,
    x_m'' = F_m'/B_m and J theta'''' = K_SE_AG x_AG'' - K_SE_ANT x_ANT''.  So
    theta(t) ~ theta''''(0) t^4/24 (Richardson-extrapolated from two small t)."""
    rng = np.random.default_rng(8)
    for _ in range(4):
        p = rand_opc(rng)
        lv = oracle.control_levels(p, 10.0)
        xa2 = (lv[2] - lv[0]) / (p[10] * 1e-3) / p[4]
        xn2 = (lv[3] - lv[1]) / (p[11] * 1e-3) / p[5]
        d4 = (p[0] * xa2 - p[1] * xn2) / p[9]
        g = []
        for t_ms in (0.1, 0.05):
            th = oracle.simulate_levels(p, lv, 2, dt_ms=t_ms, nsub=64)
            t = t_ms * 1e-3
            g.append(24 * (th[1] - th[0]) / t ** 4)
        est = 2 * g[1] - g[0]
        assert abs(est - d4) < 2e-3 * abs(d4), (est, d4)


# --- cost ----------------------------------------------------------------------------------------

def test_cost_by_hand():
    theta = np.array([0.0, 1.0])
    pos = np.array([[0.5, 0.25], [1.0, 1.0]], np.float32)
    r, m = oracle.cost(theta, pos, 90.0)       # prediction (0, theta)
    assert abs(r - math.sqrt((0.25 + 0.0625 + 1.0 + 0.0) / 4)) < 1e-12
    assert abs(m - (0.5 + 0.25 + 1.0) / 4) < 1e-12
    r1, m1 = oracle.cost(theta, pos[:, :1], 180.0)  # 1 channel, leftward: prediction -theta
    assert abs(r1 - math.sqrt((0.25 + 4.0) / 2)) < 1e-12 and abs(m1 - 1.25) < 1e-12
    rn, _ = oracle.cost(np.array([np.nan, 0.0]), pos, 0.0)
    assert rn == math.inf


# --- candidates ----------------------------------------------------------------------------------

def _nearest_f32(x: Fraction) -> np.float32:
    f = np.float32(float(x))
    best = f
    for g in (np.nextafter(f, np.float32(-np.inf)), np.nextafter(f, np.float32(np.inf))):
        dg, db = abs(Fraction(float(g)) - x), abs(Fraction(float(best)) - x)
        if dg < db or (dg == db and (int(np.float32(g).view(np.uint32)) & 1) == 0):
            best = g
    return np.float32(best)


def test_candidate_rule_exact():
    """Candidate = clamp(fl32(c + w*s)) with s = u/2^23 - 1 from the published SplitMix64
    stream; checked with exact rational arithmetic."""
    c, w, lo, hi = oracle.initial_box(43.0, 0.25)
    assert np.all(lo == np.float32(c - w)) and np.all(hi == np.float32(c + w))
    seed = 0x1234_5678_9ABC_DEF0
    for rnd, idx in [(0, 1), (0, 4095), (3, 77), (9, 65535), (1, 2**31 + 5)]:
        cand = oracle.candidate(seed, rnd, idx, c, w, lo, hi)
        for k in range(9):
            n = 1 + ((rnd << 36) | (idx << 4) | k)
            z = oracle.splitmix64(seed, n)
            for h, u in enumerate((z >> 40, (z >> 16) & 0xFFFFFF)):
                j = 2 * k + h
                s = Fraction(int(u), 2 ** 23) - 1
                v = _nearest_f32(Fraction(float(w[j])) * s + Fraction(float(c[j])))
                v = min(max(v, lo[j]), hi[j])
                assert cand[j] == v, (rnd, idx, j)
    assert np.array_equal(oracle.candidate(seed, 5, 0, c, w, lo, hi), c)


def test_candidates_fill_the_box_uniformly():
    c, w, lo, hi = oracle.initial_box(43.0, 0.25)
    X = oracle.candidates(7, 0, range(1, 4001), c, w, lo, hi).astype(np.float64)
    s = (X - c) / w
    assert np.all(X >= lo) and np.all(X <= hi)
    assert np.abs(s.mean(0)).max() < 0.06          # E[s] = 0
    assert np.abs((s ** 2).mean(0) - 1 / 3).max() < 0.03  # Var[U(-1,1)] = 1/3
    assert np.abs(np.corrcoef(s.T) - np.eye(18)).max() < 0.07


# --- search ---------------------------------------------------------------------------------------

def test_fit_recovers_truth_in_candidate_set():
    """Noise-free target made from candidate 37 of round 0: the argmin is 37 and its RMSE is
    only the FP32 rounding of the trace."""
    seed = 99
    c, w, lo, hi = oracle.initial_box(43.0, 0.25)
    truth = oracle.candidate(seed, 0, 37, c, w, lo, hi)
    pos = oracle.make_target(truth.astype(np.float64), 10.0, 0.0, 80, 1, np.zeros((80, 1)), 0.0)
    res = oracle.fit(pos, 10.0, 0.0, 43.0, seed, 200, 1, nthreads=4)
    assert res["best_idx"][0] == 37
    assert res["rmse"] < 2e-7
    assert np.array_equal(res["opc"], truth)


def test_fit_monotone_and_ties():
    b = synth.draw_saccades(1, "tiny")
    p = oracle.true_opc(b["mult"][0], 43.0)
    pos = oracle.make_target(p, 10.0, 0.0, 80, 1, b["noise"][0], 0.05)
    res = oracle.fit(pos, 10.0, 0.0, 43.0, int(b["seed"][0]), 64, 5, nthreads=4)
    br = res["best_rmse"]
    assert np.all(np.diff(br) <= 0)
    # every round is centred on the previous winner
    c, w, lo, hi = oracle.initial_box(43.0, 0.25)
    cen = res["centres"]
    for r in range(1, 5):
        ww = w * np.float32(0.5 ** (r - 1))
        prev = oracle.candidate(int(b["seed"][0]), r - 1, int(res["best_idx"][r - 1]), cen[r - 1], ww, lo, hi)
        assert np.array_equal(prev, cen[r])
    # zero half-width: every candidate is the centre; ties go to index 0
    res0 = oracle.fit(pos, 10.0, 0.0, 43.0, 5, 16, 1, w_init_frac=0.0)
    assert res0["best_idx"][0] == 0


def test_brute_force_grid():
    """Exhaustive 5x5x5 grid over (N_SAC_AG, tau_AC_AG, PW) with the truth on the grid and a
    noise-free target: the grid argmin is the truth, and the threaded scorer agrees with a
    per-candidate serial loop."""
    base = oracle.nominal(43.0).astype(np.float32)
    levels = {15: [45, 50, 55, 60, 65], 10: [9.5, 10.6, 11.7, 12.8, 13.9], 17: [33, 35, 37, 39, 41]}
    grid = []
    for a in levels[15]:
        for b in levels[10]:
            for c_ in levels[17]:
                q = base.copy(); q[15] = a; q[10] = b; q[17] = c_
                grid.append(q)
    grid = np.array(grid, np.float32)
    truth_i = 2 * 25 + 3 * 5 + 1
    pos = oracle.make_target(grid[truth_i].astype(np.float64), 10.0, 0.0, 80, 1, np.zeros((80, 1)), 0.0)
    r, _ = oracle.score(grid, pos, 10.0, 0.0, nthreads=4)
    assert int(np.argmin(r)) == truth_i and r[truth_i] < 2e-7
    for i in (0, 17, truth_i, 124):
        th = oracle.simulate(grid[i].astype(np.float64), 10.0, 80)
        assert oracle.cost(th, pos, 0.0)[0] == r[i]


def test_model9_stream_and_truth_recovery():
    """9-parameter model (Section 2.2.2, Table 2): one K_SE and one K_LT for both muscles, the
    neuronal-control parameters at nominal; a noise-free target made from one of its candidates is
    recovered exactly."""
    c, w, lo, hi = oracle.initial_box(43.0, 0.25, model=9)
    fixed = [10, 11, 12, 13, 15, 16, 17]
    assert np.all(w[fixed] == 0) and np.all(w[[0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 14]] > 0)
    X = oracle.candidates(3, 0, range(1, 200), c, w, lo, hi, model=9)
    assert np.all(X[:, 1] == X[:, 0]) and np.all(X[:, 3] == X[:, 2])
    assert np.all(X[:, fixed] == c[fixed])
    truth = oracle.candidates(77, 0, [41], c, w, lo, hi, model=9)[0]
    pos = oracle.make_target(truth.astype(np.float64), 10.0, 0.0, 80, 1, np.zeros((80, 1)), 0.0)
    res = oracle.fit(pos, 10.0, 0.0, 43.0, 77, 100, 1, model=9, nthreads=4)
    assert res["best_idx"][0] == 41 and np.array_equal(res["opc"], truth)


# --- the paper's estimator: Nelder-Mead (Section 3.3) ---------------------------------------------

def _nm_problem(seed=5, noise=0.0):
    rng = np.random.default_rng(seed)
    dur, amp = 43.0, 10.0
    p_true = oracle.nominal(dur) * rng.uniform(0.95, 1.05, 18)
    T = 80
    th = oracle.simulate(p_true, amp, T)
    pos = (th + noise * rng.standard_normal(T)).astype(np.float32)[:, None]
    return pos, amp, dur


def _rmse_at(x_rel, pos, amp, dur, lo=0.75, hi=1.25):
    p = np.float32(np.clip(x_rel, lo, hi) * oracle.nominal(dur)).astype(np.float64)
    return oracle.cost(oracle.simulate(p, amp, pos.shape[0]), pos, 0.0)[0]


def test_nelder_mead_exit_needs_both_tolerances():
    """The initial simplex (x0 and x0 with one coordinate scaled by 1.05) spreads 0.05 in x and some
    amount in f: loose tolerances on both stop at once, one tight tolerance keeps it going."""
    pos, amp, dur = _nm_problem()
    assert oracle.nelder_mead(pos, amp, 0.0, dur, max_iter=50, tol_x=1.0, tol_f=1.0)["iters"] == 0
    assert oracle.nelder_mead(pos, amp, 0.0, dur, max_iter=50, tol_x=1.0, tol_f=1e-12)["iters"] > 0
    assert oracle.nelder_mead(pos, amp, 0.0, dur, max_iter=50, tol_x=0.01, tol_f=1.0)["iters"] > 0


def test_nelder_mead_initial_simplex_best_vertex():
    """Stopped before the first iteration, the result is the best of the 19 initial vertices."""
    pos, amp, dur = _nm_problem()
    r = oracle.nelder_mead(pos, amp, 0.0, dur, max_iter=0)
    verts = [np.ones(18)] + [np.where(np.arange(18) == j, 1.05, 1.0) for j in range(18)]
    costs = [_rmse_at(v, pos, amp, dur) for v in verts]
    best = int(np.argmin(costs))
    assert np.array_equal(r["opc"], np.float32(verts[best] * oracle.nominal(dur)))
    assert abs(r["rmse"] - costs[best]) <= 1e-12


def test_nelder_mead_descends_and_replays_itself():
    """On a noise-free target 5% from nominal the simplex search lowers the RMSE by orders of
    magnitude, its best value never rises, and replaying its own decisions reproduces it exactly."""
    pos, amp, dur = _nm_problem()
    r0 = _rmse_at(np.ones(18), pos, amp, dur)
    r = oracle.nelder_mead(pos, amp, 0.0, dur, max_iter=1500, tol_x=0.0, tol_f=0.0)
    assert r["rmse"] < 1e-2 * r0, (r["rmse"], r0)
    assert set(np.unique(r["own"])) <= {0, 1, 2, 3, 4}
    short = [oracle.nelder_mead(pos, amp, 0.0, dur, max_iter=n, tol_x=0.0, tol_f=0.0)["rmse"] for n in (50, 200, 800)]
    assert short[0] >= short[1] >= short[2] >= r["rmse"]
    again = oracle.nelder_mead(pos, amp, 0.0, dur, max_iter=1500, tol_x=0.0, tol_f=0.0, forced=r["own"])
    assert np.array_equal(again["opc"], r["opc"]) and again["rmse"] == r["rmse"]


def test_nelder_mead_steps_follow_lagarias():
    """The first iterations, rebuilt here from the transformation's definition (Lagarias et al.
    1998: reflection 1, expansion 2, contractions 1/2, shrink 1/2, the simplex sorted stably after
    each step): every decision and the best vertex agree, and the runs exercise every kind of step
    (the last case is one whose 263rd step is a shrink)."""
    seen = set()
    for seed, noise, n_it in ((0, 0.05, 40), (1, 0.05, 40), (2, 0.05, 40), (3, 0.05, 40), (9, 0.5, 300)):
        pos, amp, dur = _nm_problem(seed=seed, noise=noise)
        cache = {}

        def f(x):
            k = tuple(np.round(x, 15))
            if k not in cache:
                cache[k] = _rmse_at(x, pos, amp, dur)
            return cache[k]
        V = [np.ones(18)] + [np.where(np.arange(18) == j, 1.05, 1.0) for j in range(18)]
        F = [f(v) for v in V]
        r = oracle.nelder_mead(pos, amp, 0.0, dur, max_iter=n_it, tol_x=0.0, tol_f=0.0)
        for it in range(n_it):
            order = np.argsort(F, kind="stable")
            V = [V[i] for i in order]
            F = [F[i] for i in order]
            xb = np.mean(V[:18], axis=0)
            w = V[18]
            pt = [xb + (xb - w), xb + 2 * (xb - w), xb + 0.5 * (xb - w), xb - 0.5 * (xb - w)]
            fr = f(pt[0])
            if fr < F[0]:
                d = 1 if f(pt[1]) < fr else 0
            elif fr < F[17]:
                d = 0
            elif fr < F[18]:
                d = 2 if f(pt[2]) <= fr else 4
            else:
                d = 3 if f(pt[3]) < F[18] else 4
            assert r["own"][it] == d, (seed, it, r["own"][it], d)
            seen.add(d)
            if d < 4:
                V[18], F[18] = pt[d], f(pt[d])
            else:
                V = [V[0]] + [V[0] + 0.5 * (v - V[0]) for v in V[1:]]
                F = [F[0]] + [f(v) for v in V[1:]]
        best = V[int(np.argsort(F, kind="stable")[0])]
        assert np.array_equal(r["opc"], np.float32(np.clip(best, 0.75, 1.25) * oracle.nominal(dur))), seed
    assert seen >= {0, 1, 2, 3, 4}, seen


# --- regression anchor: numbers computed independently for the nominal plant ---------------------

def _anchor_rows():
    rows = {}
    for line in open(os.path.join(GOLD, "anchor_nominal_10deg.txt")):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            rows.setdefault(k, []).append([float(x) for x in v])
    return rows


def anchor_trajectory_errors(simulate):
    """Largest deviations of a simulator from the anchor: (theta error in deg, peak-velocity error in
    deg/s).  `simulate(p, amp, T, dt_ms)` returns theta at t_k = k dt_ms."""
    rows = _anchor_rows()
    p = oracle.nominal(43.0)
    th = simulate(p, 10.0, 80, 1.0)
    err = max(abs(th[int(t)] - v) for t, v in rows["theta"])
    fine = simulate(p, 10.0, 800, 0.1)
    vmax = float(np.max(np.diff(fine))) / 1e-4
    return err, abs(vmax - rows["peak_velocity"][0][0])


def test_anchor_nominal_trajectory():
    """Nominal OPC, A = 10 deg, D = 43 ms: theta at 10..79 ms to the anchor's three decimals and the
    peak velocity to ~1 deg/s (independent numbers for the same model reading)."""
    err, verr = anchor_trajectory_errors(lambda p, a, T, dt: oracle.simulate(p, a, T, dt_ms=dt))
    assert err <= 5e-4 + 1e-12, err
    assert verr < 1.0, verr


def anchor_eigen_errors(rhs):
    """Worst relative deviation of the eigenvalues of each piece's system matrix from the anchor.
    `rhs(p, x, n_ag, n_ant, tau_ag_s, tau_ant_s)` is the plant's right-hand side (1/s units)."""
    rows = _anchor_rows()

    def eig(p, n_ag, n_ant, ta, tn):
        b = rhs(p, np.zeros(6), n_ag, n_ant, ta, tn)
        A = np.zeros((6, 6))
        for j in range(6):
            e = np.zeros(6); e[j] = 1.0
            A[:, j] = rhs(p, e, n_ag, n_ant, ta, tn) - b
        ev = np.linalg.eigvals(A)
        return np.sort(ev.real), float(np.abs(ev.imag).max())

    worst = 0.0
    p = oracle.nominal(43.0)
    lv = oracle.control_levels(p, 10.0)
    for piece, (n_ag, n_ant, ta, tn) in (("act_pulse", (lv[2], lv[3], p[10] * 1e-3, p[11] * 1e-3)),
                                         ("act_post", (lv[4], lv[5], p[12] * 1e-3, p[13] * 1e-3))):
        ev, im = eig(p, n_ag, n_ant, ta, tn)
        worst = max(worst, im)
        for want in rows[piece][0]:      # -1/tau of each active state is an eigenvalue
            worst = max(worst, np.min(np.abs(ev - want)) / abs(want))
    q = p.copy(); q[7] = 0.0             # K_P = N_C_ANT = 0.5 g/deg
    ev, im = eig(q, lv[2], lv[3], p[10] * 1e-3, p[11] * 1e-3)
    want = np.sort(np.array(rows["mech_kp0.5"][0] + rows["act_pulse"][0]))
    worst = max(worst, im, float(np.max(np.abs(ev - want) / np.abs(want))))
    return worst


def test_anchor_eigenvalues():
    """Eigenvalues of the pulse and post system matrices (probed from the plant's right-hand side)
    against the anchor to 0.1 %: the activation modes -1/tau in each piece, and the four mechanical
    modes (shared by both pieces) at the anchor's passive elasticity."""
    assert anchor_eigen_errors(oracle.rhs) < 1e-3


def test_seeded_round0_centre():
    """A seeded fit starts at the seed clamped into the box; a NaN component keeps the nominal centre
    (the library's documented rule for an unusable seed); with one candidate per round (the centre)
    nothing moves, so the reported OPC is that start."""
    c0, w0, lo, hi = oracle.initial_box(43.0)
    seed = (c0 * np.float32(1.1)).astype(np.float32)
    seed[4] = hi[4] * np.float32(2.0)
    seed[7] = np.nan
    pos = np.zeros((80, 1), np.float32)
    res = oracle.fit(pos, 10.0, 0.0, 43.0, 5, 1, 2, w_init_frac=0.25, c_init=seed)
    want = np.where(np.isnan(seed), c0, np.minimum(np.maximum(seed, lo), hi)).astype(np.float32)
    assert want[4] == hi[4] and want[7] == c0[7]
    assert np.array_equal(res["centres"][0], want) and np.array_equal(res["opc"], want)
