"""OPMM oracle -- test infrastructure only.

A plain, serial FP64 CPU implementation (``opmm_oracle.c``) of what the OPMM
estimation path computes, plus the plain numpy reference for the surrogate MLP
(``mlp_ref``).  Only the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU path and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "opmm_oracle.c")
_SO = os.path.join(_HERE, "libopmm_oracle.so")
_SAN_SO = os.path.join(_HERE, "libopmm_oracle_san.so")
# OPMM_ORACLE_SANITIZE=1 loads the build instrumented with AddressSanitizer and UndefinedBehaviorSanitizer
# (the process must then start with the ASan runtime preloaded; tests/test_oracle_sanitized.py does this)
_SANITIZE = os.environ.get("OPMM_ORACLE_SANITIZE") == "1"
NP_ = 18

_FLAGS = ["-std=c11", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra", "-shared", "-fPIC"]


def build(force: bool = False, sanitize: bool = None) -> str:
    """Compile the C oracle with gcc: FP64, no fast-math, no FMA contraction.  sanitize (default: the
    OPMM_ORACLE_SANITIZE setting): the ASan + UBSan build, every finding fatal."""
    sanitize = _SANITIZE if sanitize is None else sanitize
    so = _SAN_SO if sanitize else _SO
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(_SRC):
        tmp = so + ".tmp%d" % os.getpid()
        opt = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer"] if sanitize else ["-O2"]
        subprocess.check_call(["gcc"] + opt + _FLAGS + ["-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, so)
    return so


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        d, i, f = ctypes.c_double, ctypes.c_int, ctypes.c_float
        P = ctypes.c_void_p
        u64, i64, u32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32
        L.oracle_nominal.argtypes = [d, P]
        L.oracle_rhs.argtypes = [P, P, d, d, d, d, P]
        L.oracle_equilibrium.argtypes = [P, d, d, P]
        L.oracle_control_levels.argtypes = [P, d, P]
        L.oracle_simulate_levels.argtypes = [P, P, i, d, i, P, P]
        L.oracle_simulate_levels.restype = i
        L.oracle_simulate.argtypes = [P, d, i, d, i, P]
        L.oracle_simulate.restype = i
        L.oracle_cost.argtypes = [P, P, i, i, d, P, P]
        L.oracle_splitmix64.argtypes = [u64, u64]
        L.oracle_splitmix64.restype = u64
        L.oracle_candidate.argtypes = [u64, u32, u32, P, P, P, P, P]
        L.oracle_initial_box.argtypes = [d, f, P, P, P, P]
        L.oracle_score.argtypes = [P, i64, P, i, i, d, d, d, i, i, P, P]
        L.oracle_score.restype = i
        L.oracle_fit.argtypes = [P, i, i, d, d, d, d, u64, i64, i, f, f, f, P, i, i, i,
                                 P, P, P, P, P, P]
        L.oracle_initial_box_model.argtypes = [d, f, i, P, P, P, P]
        L.oracle_tie_model9.argtypes = [P]
        L.oracle_fit.restype = i
        L.oracle_nelder_mead.argtypes = [P, i, i, d, d, d, d, P, i, d, d, d, d, i, P, P, P, P, P]
        L.oracle_nelder_mead.restype = i
        L.oracle_jacobian.argtypes = [P, d, i, d, i, d, P, P]
        L.oracle_jacobian.restype = i
        L.oracle_damped_solve.argtypes = [i, P, P, d, P, P]
        L.oracle_damped_solve.restype = i
        L.oracle_polish.argtypes = [P, i, i, d, d, d, d, P, i, i, i, d, d, d, i, d, P, P, P, P, P, P]
        L.oracle_polish.restype = i
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.shape == (n,), a.shape
    return a


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


NSUB = 16  # RK4 substeps per sample


def nominal(dur_ms: float) -> np.ndarray:
    out = np.zeros(NP_)
    lib().oracle_nominal(float(dur_ms), _p(out))
    return out


def rhs(p, x, n_ag, n_ant, tau_ag, tau_ant) -> np.ndarray:
    p = _f64(p, NP_); x = _f64(x, 6); dx = np.zeros(6)
    lib().oracle_rhs(_p(p), _p(x), n_ag, n_ant, tau_ag, tau_ant, _p(dx))
    return dx


def equilibrium(p, f_ag, f_ant) -> np.ndarray:
    p = _f64(p, NP_); x = np.zeros(6)
    lib().oracle_equilibrium(_p(p), float(f_ag), float(f_ant), _p(x))
    return x


def control_levels(p, amp) -> np.ndarray:
    p = _f64(p, NP_); lv = np.zeros(6)
    lib().oracle_control_levels(_p(p), float(amp), _p(lv))
    return lv


def simulate_levels(p, levels, T, dt_ms=1.0, nsub=NSUB, states=False):
    p = _f64(p, NP_); lv = _f64(levels, 6)
    th = np.zeros(max(T, 1)); st = np.zeros((max(T, 1), 6)) if states else None
    rc = lib().oracle_simulate_levels(_p(p), _p(lv), int(T), float(dt_ms), int(nsub), _p(th),
                                      _p(st) if states else None)
    assert rc == 0
    return (th[:T], st[:T]) if states else th[:T]


def simulate(p, amp, T, dt_ms=1.0, nsub=NSUB) -> np.ndarray:
    p = _f64(p, NP_); th = np.zeros(max(T, 1))
    assert lib().oracle_simulate(_p(p), float(amp), int(T), float(dt_ms), int(nsub), _p(th)) == 0
    return th[:T]


def cost(theta, pos, dir_deg):
    theta = _f64(theta); pos = _f32(pos)
    T = theta.shape[0]; C = pos.shape[1]
    assert pos.shape == (T, C)
    r = ctypes.c_double(); m = ctypes.c_double()
    lib().oracle_cost(_p(theta), _p(pos), T, C, float(dir_deg), ctypes.byref(r), ctypes.byref(m))
    return r.value, m.value


def splitmix64(seed: int, n: int) -> int:
    return int(lib().oracle_splitmix64(ctypes.c_uint64(seed), ctypes.c_uint64(n)))


def initial_box(dur_ms, frac=0.25, model=18):
    c, w, lo, hi = (np.zeros(NP_, np.float32) for _ in range(4))
    lib().oracle_initial_box_model(float(dur_ms), ctypes.c_float(frac), int(model), _p(c), _p(w), _p(lo), _p(hi))
    return c, w, lo, hi


def tie_model9(p):
    """The 9-parameter model's ties applied to a candidate (copy)."""
    q = np.array(p, np.float32)
    lib().oracle_tie_model9(_p(q))
    return q


def candidate(seed, rnd, idx, c, w, lo, hi) -> np.ndarray:
    out = np.zeros(NP_, np.float32)
    c, w, lo, hi = (_f32(a) for a in (c, w, lo, hi))
    lib().oracle_candidate(ctypes.c_uint64(seed), rnd, idx, _p(c), _p(w), _p(lo), _p(hi), _p(out))
    return out


def candidates(seed, rnd, idxs, c, w, lo, hi, model=18) -> np.ndarray:
    out = np.stack([candidate(seed, rnd, int(i), c, w, lo, hi) for i in idxs])
    if model == 9:
        out[:, 1] = out[:, 0]
        out[:, 3] = out[:, 2]
    return out


def score(opc, pos, amp, dir_deg, dt_ms=1.0, nsub=NSUB, nthreads=1):
    """RMSE and mean-abs of each FP32 candidate (promoted to FP64) against one saccade."""
    opc = _f32(opc).reshape(-1, NP_); pos = _f32(pos)
    n = opc.shape[0]; T, C = pos.shape
    r = np.zeros(n); m = np.zeros(n)
    assert lib().oracle_score(_p(opc), n, _p(pos), T, C, float(amp), float(dir_deg), float(dt_ms),
                              nsub, int(nthreads), _p(r), _p(m)) == 0
    return r, m


def fit(pos, amp, dir_deg, dur_ms, seed, n_cand, n_rounds, *, dt_ms=1.0, box_frac=0.25,
        w_init_frac=1.0, shrink=0.5, c_init=None, model=18, nsub=NSUB, nthreads=1):
    pos = _f32(pos); T, C = pos.shape
    opc = np.zeros(NP_, np.float32); rm = ctypes.c_double(); ma = ctypes.c_double()
    bi = np.zeros(n_rounds, np.int64); br = np.zeros(n_rounds); cen = np.zeros((n_rounds, NP_), np.float32)
    ci = None if c_init is None else _f32(c_init)
    rc = lib().oracle_fit(_p(pos), T, C, float(amp), float(dir_deg), float(dur_ms), float(dt_ms),
                          ctypes.c_uint64(seed), int(n_cand), int(n_rounds), ctypes.c_float(box_frac),
                          ctypes.c_float(w_init_frac), ctypes.c_float(shrink),
                          None if ci is None else _p(ci), int(model), nsub, int(nthreads), _p(opc),
                          ctypes.byref(rm), ctypes.byref(ma), _p(bi), _p(br), _p(cen))
    assert rc == 0
    return dict(opc=opc, rmse=rm.value, mae=ma.value, best_idx=bi, best_rmse=br, centres=cen)


def true_opc(mult, dur_ms) -> np.ndarray:
    """A synthetic 'true' OPC: the Table 1 nominal scaled component-wise."""
    return nominal(dur_ms) * np.asarray(mult, np.float64)


def make_target(p_true, amp, dir_deg, T, C, noise_z, sigma):
    """Recorded-trace stand-in: the plant's prediction along the direction plus
    Gaussian noise, built in FP64 and rounded once to FP32, [T][C]."""
    th = simulate(p_true, amp, T)
    phi = np.deg2rad(dir_deg)
    u = np.array([np.cos(phi), np.sin(phi)])[:C]
    pos = th[:, None] * u[None, :] + sigma * np.asarray(noise_z, np.float64).reshape(T, C)
    return pos.astype(np.float32)


def nelder_mead(pos, amp, dir_deg, dur_ms, *, x0=None, max_iter=500, tol_x=1e-4, tol_f=1e-6, lo=0.75, hi=1.25,
                dt_ms=1.0, nsub=NSUB, forced=None):
    """The paper's Nelder-Mead (Lagarias variant) on the RMSE.  Returns dict(opc, rmse, iters, own, margin):
    own/margin per iteration = the oracle's own decision and the smallest gap it rested on; with forced
    (decision codes) the run follows those decisions instead."""
    pos = _f32(pos); T, C = pos.shape
    opc = np.zeros(NP_, np.float32); f = ctypes.c_double()
    own = np.full(max(max_iter, 1), -1, np.int8); mar = np.zeros(max(max_iter, 1))
    x0p = None if x0 is None else _p(_f32(x0))
    fc = None
    if forced is not None:
        fc = np.zeros(max(max_iter, 1), np.int8)
        fc[:len(forced)] = forced
    it = lib().oracle_nelder_mead(_p(pos), T, C, float(amp), float(dir_deg), float(dur_ms), float(dt_ms), x0p,
                                  int(max_iter), float(tol_x), float(tol_f), float(lo), float(hi), int(nsub),
                                  None if fc is None else _p(fc), _p(own), _p(mar), _p(opc), ctypes.byref(f))
    return dict(opc=opc, rmse=f.value, iters=it, own=own[:it], margin=mar[:it])


def jacobian(p, amp, T, dt_ms=1.0, nsub=NSUB, h_rel=3e-5):
    """(theta [T], d theta / d p [T][18]) by central differences of the RK4 trajectory."""
    p = np.ascontiguousarray(p, np.float64)
    th = np.zeros(T); J = np.zeros((T, NP_))
    rc = lib().oracle_jacobian(_p(p), float(amp), int(T), float(dt_ms), int(nsub), float(h_rel), _p(th), _p(J))
    assert rc == 0
    return th, J


def damped_solve(H, g, lam, held=None):
    """delta solving (H + lam diag H) delta = -g (held unknowns: 0), or None if not positive definite."""
    H = np.ascontiguousarray(H, np.float64); g = np.ascontiguousarray(g, np.float64)
    n = g.shape[0]
    hd = np.ascontiguousarray(np.zeros(n, np.int32) if held is None else held, np.int32)
    dl = np.zeros(n)
    rc = lib().oracle_damped_solve(n, _p(H), _p(g), float(lam), _p(hd), _p(dl))
    return None if rc != 0 else dl


def polish(pos, amp, dir_deg, dur_ms, x0, *, model=18, objective=0, max_iter=20, tol_f=1e-10, lam0=1e-3,
           box_frac=0.25, dt_ms=1.0, nsub=NSUB, forced=None, h_rel=3e-5):
    """Levenberg-Marquardt polish (objective 0: sum of squares, 1: sum of absolute differences), the
    Jacobian by central differences with step h_rel |p_j|.  Returns dict(opc, f, iters, own, margin,
    fhist); with forced, exactly len(forced) iterations following those decisions."""
    pos = _f32(pos); T, C = pos.shape
    x0 = _f32(x0)
    n = max_iter if forced is None else len(forced)
    own = np.full(max(n, 1), -2, np.int8); mar = np.zeros(max(n, 1)); fh = np.zeros(max(n, 1))
    fc = None if forced is None else np.ascontiguousarray(forced, np.int8)
    opc = np.zeros(NP_, np.float32); f = ctypes.c_double()
    it = lib().oracle_polish(_p(pos), T, C, float(amp), float(dir_deg), float(dur_ms), float(dt_ms), _p(x0),
                             int(model), int(objective), int(n), float(tol_f), float(lam0), float(box_frac),
                             int(nsub), float(h_rel), None if fc is None else _p(fc), _p(own), _p(mar), _p(fh), _p(opc),
                             ctypes.byref(f))
    return dict(opc=opc, f=f.value, iters=it, own=own[:it], margin=mar[:it], fhist=fh[:it])


def ivt(gaze, dt_ms=1.0, vel_thresh=30.0, min_dur=6.0, min_amp=0.0, max_T=2048):
    """I-VT written as plain loops (Section 3.1 / Section 4: velocity-threshold identification, short
    saccades dropped).  A sample k >= 1 is fast when |g_k - g_(k-1)| / dt > threshold (compared
    squared, per sample, in FP32 like the stream's own values); a saccade is a maximal run of fast
    samples plus the fixation sample before it, re-based to that sample.  Returns a list of dicts
    (start = index of the prepended sample, T, amp, dir, trace [T][2] float32)."""
    g = np.asarray(gaze, np.float32)
    N = g.shape[0]
    v = np.float32(vel_thresh) * np.float32(dt_ms) * np.float32(1e-3)
    thr2 = v * v

    def fast(k):
        dx = g[k, 0] - g[k - 1, 0]
        dy = g[k, 1] - g[k - 1, 1]
        return dx * dx + dy * dy > thr2

    out = []
    k = 1
    while k < N:
        if fast(k):
            k0 = k
            while k + 1 < N and fast(k + 1):
                k += 1
            k1 = k
            T = k1 - k0 + 2
            d = g[k1] - g[k0 - 1]
            amp = float(np.sqrt(np.float32(d[0] * d[0] + d[1] * d[1])))
            ang = float(np.degrees(np.arctan2(float(d[1]), float(d[0]))))
            if ang < 0:
                ang += 360.0
            if (T - 1) * dt_ms >= min_dur and amp >= min_amp and T <= max_T:
                out.append(dict(start=k0 - 1, T=T, amp=amp, dir=ang, trace=(g[k0 - 1:k1 + 1] - g[k0 - 1])))
        k += 1
    return out
