"""Thin Python binding of libopmm (include/opmm.h).

Argument marshalling only: every step of the estimation path runs in the HIP
kernels of libopmm.so.  Tensors are torch CUDA tensors (device memory and the
current stream are all PyTorch is used for).  If the library is not built the
import of this module fails: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("OPMM_LIBRARY") or os.path.join(_PKG, "libopmm.so")
P = 18
MAX_T = 2048

OK, EINVAL, ENOMEM, EDEVICE, ENOTREADY = 0, -1, -2, -3, -4
ST_OK, ST_NONFINITE_INPUT, ST_NO_FINITE_CANDIDATE, ST_SEEDED, ST_FALLBACK, ST_WAIT_TIMEOUT, ST_DEADLINE = \
    0, 1, 2, 4, 8, 16, 32
FIT_ROUNDS, FIT_PERSISTENT = 0, 1
KERNEL_ROUND, KERNEL_SCREEN, KERNEL_VERIFY, KERNEL_PERSISTENT = 0, 1, 2, 3

SACCADE_DTYPE = np.dtype([("pos_offset", "<i8"), ("T", "<i4"), ("C", "<i4"), ("amp_deg", "<f4"),
                          ("dir_deg", "<f4"), ("dur_ms", "<f4"), ("n_cand", "<i4"), ("seed", "<u8")])
assert SACCADE_DTYPE.itemsize == 40


class FitParams(ctypes.Structure):
    _fields_ = [("n_cand", ctypes.c_int32), ("n_rounds", ctypes.c_int32), ("box_frac", ctypes.c_float),
                ("w_init_frac", ctypes.c_float), ("shrink", ctypes.c_float), ("dt_ms", ctypes.c_float),
                ("mode", ctypes.c_int32), ("tile", ctypes.c_int32), ("model", ctypes.c_int32),
                ("screen_rounds", ctypes.c_int32), ("screen_tol", ctypes.c_float)]


class ServeParams(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("max_T", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_size_t),
                ("plain", FitParams), ("seeded", FitParams), ("fallback_rmse", ctypes.c_float),
                ("polish_iter", ctypes.c_int32), ("rounds_per_step", ctypes.c_int32)]


class NmParams(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("tol_x", ctypes.c_float), ("tol_f", ctypes.c_float),
                ("box_frac", ctypes.c_float), ("dt_ms", ctypes.c_float), ("max_ms", ctypes.c_float),
                ("tasks_per_wave", ctypes.c_int32)]


class PolishParams(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("objective", ctypes.c_int32), ("tol_f", ctypes.c_float),
                ("lambda0", ctypes.c_float), ("box_frac", ctypes.c_float), ("dt_ms", ctypes.c_float)]


OBJ_RMSE, OBJ_MAE = 0, 1


class OpmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("opmm error %d: %s" % (code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libopmm.so is not built (run __graft_entry__.build()); there is no fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64, f = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                 ctypes.c_uint64, ctypes.c_float)
    sig = {
        "opmm_fit_params_default": (None, [ctypes.POINTER(FitParams)]),
        "opmm_nominal": (None, [f, vp]),
        "opmm_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int]),
        "opmm_destroy": (ctypes.c_int, [vp]),
        "opmm_last_error": (ctypes.c_char_p, [vp]),
        "opmm_set_wait_limit": (ctypes.c_int, [vp, u32]),
        "opmm_sync": (ctypes.c_int, [vp, vp]),
        "opmm_kernel_timing_enable": (ctypes.c_int, [vp, i32]),
        "opmm_kernel_timing_read": (ctypes.c_int, [vp, i32, ctypes.POINTER(ctypes.c_double),
                                                   ctypes.POINTER(ctypes.c_int64)]),
        "opmm_candidates": (ctypes.c_int, [vp, u64, u32, u32, i64, vp, vp, vp, vp, vp, vp]),
        "opmm_simulate": (ctypes.c_int, [vp, vp, vp, i64, i32, f, vp, vp]),
        "opmm_score": (ctypes.c_int, [vp, vp, i64, vp, i64, vp, f, vp, vp]),
        "opmm_score_screen": (ctypes.c_int, [vp, vp, i64, vp, i64, vp, f, vp, vp]),
        "opmm_fit": (ctypes.c_int, [vp, vp, i64, vp, i32, ctypes.POINTER(FitParams), vp, vp, vp, vp, vp,
                                    vp, vp]),
        "opmm_fit_noalloc": (ctypes.c_int, [vp, vp, i64, vp, i32, ctypes.POINTER(FitParams), vp, vp, vp, vp, vp,
                                            vp, vp]),
        "opmm_fit_plan_create": (ctypes.c_int, [vp, vp, i64, vp, i32, ctypes.POINTER(FitParams), vp, vp,
                                                vp, vp, vp, vp, vp, ctypes.POINTER(vp)]),
        "opmm_plan_launch": (ctypes.c_int, [vp, vp]),
        "opmm_plan_destroy": (ctypes.c_int, [vp]),
        "opmm_autotune": (ctypes.c_int, [vp, vp, i64, vp, i32, ctypes.POINTER(FitParams),
                                         ctypes.POINTER(i32), vp]),
        "opmm_tune_cache_lookup": (ctypes.c_int, [vp, vp, i32, ctypes.POINTER(FitParams), ctypes.POINTER(i32)]),
        "opmm_tune_cache_save": (ctypes.c_int, [vp, ctypes.c_char_p]),
        "opmm_tune_cache_load": (ctypes.c_int, [vp, ctypes.c_char_p]),
        "opmm_tile_count": (ctypes.c_int, []),
        "opmm_tile_default": (ctypes.c_int, []),
        "opmm_tile_name": (ctypes.c_char_p, [ctypes.c_int]),
        "opmm_surrogate_create": (ctypes.c_int, [vp, u64, ctypes.POINTER(vp)]),
        "opmm_surrogate_destroy": (ctypes.c_int, [vp]),
        "opmm_surrogate_param_count": (i64, []),
        "opmm_surrogate_get_params": (ctypes.c_int, [vp, ctypes.c_int, vp]),
        "opmm_surrogate_set_params": (ctypes.c_int, [vp, vp]),
        "opmm_surrogate_forward": (ctypes.c_int, [vp, vp, i32, vp, vp]),
        "opmm_surrogate_backward": (ctypes.c_int, [vp, vp, vp, i32, vp, vp]),
        "opmm_surrogate_adam_step": (ctypes.c_int, [vp, f, vp]),
        "opmm_surrogate_generate": (ctypes.c_int, [vp, u64, u64, i32, f, f, vp, vp, vp]),
        "opmm_surrogate_train": (ctypes.c_int, [vp, u64, i32, i32, f, f, f, f, vp, vp]),
        "opmm_surrogate_features": (ctypes.c_int, [vp, vp, i64, vp, i32, f, vp, vp]),
        "opmm_surrogate_predict": (ctypes.c_int, [vp, vp, i64, vp, i32, f, f, vp, vp]),
        "opmm_surrogate_save": (ctypes.c_int, [vp, ctypes.c_char_p]),
        "opmm_serve_params_default": (None, [ctypes.POINTER(ServeParams)]),
        "opmm_nm_params_default": (None, [ctypes.POINTER(NmParams)]),
        "opmm_ivt_extract": (ctypes.c_int, [vp, vp, i64, f, f, f, f, i32, u64, i32, vp, vp, i64, vp,
                                            ctypes.POINTER(i32), vp]),
        "opmm_fit_nm": (ctypes.c_int, [vp, vp, i64, vp, i32, ctypes.POINTER(NmParams), vp, vp, vp, vp, vp, vp,
                                       vp]),
        "opmm_server_create": (ctypes.c_int, [vp, vp, ctypes.POINTER(ServeParams), ctypes.POINTER(vp)]),
        "opmm_server_destroy": (ctypes.c_int, [vp]),
        "opmm_server_slots": (ctypes.c_int, [vp]),
        "opmm_server_now": (ctypes.c_double, []),
        "opmm_server_submit": (ctypes.c_int, [vp, vp, vp, ctypes.c_double, ctypes.POINTER(i64)]),
        "opmm_server_step": (ctypes.c_int, [vp, ctypes.POINTER(i32)]),
        "opmm_server_submit_many": (ctypes.c_int, [vp, vp, i64, vp, i32, vp, vp]),
        "opmm_server_poll": (ctypes.c_int, [vp, i64, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i64)]),
        "opmm_server_stats": (ctypes.c_int, [vp, vp]),
        "opmm_fit_learned": (ctypes.c_int, [vp, vp, i64, vp, i32, ctypes.POINTER(FitParams),
                                            ctypes.POINTER(FitParams), f, vp, vp, vp, vp, ctypes.POINTER(i32), vp]),
        "opmm_surrogate_load": (ctypes.c_int, [vp, ctypes.c_char_p]),
        "opmm_polish_params_default": (None, [ctypes.POINTER(PolishParams)]),
        "opmm_sensitivity": (ctypes.c_int, [vp, vp, i32, vp, f, vp, vp, vp]),
        "opmm_polish": (ctypes.c_int, [vp, vp, i64, vp, i32, ctypes.POINTER(PolishParams), i32, vp, vp, vp, vp,
                                       vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def fit_params(**kw) -> FitParams:
    p = FitParams()
    lib.opmm_fit_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError("unknown fit parameter %r" % k)
        setattr(p, k, v)
    return p


def polish_params(**kw) -> PolishParams:
    p = PolishParams()
    lib.opmm_polish_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError("unknown polish parameter %r" % k)
        setattr(p, k, v)
    return p


def nm_params(**kw) -> NmParams:
    p = NmParams()
    lib.opmm_nm_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError("unknown Nelder-Mead parameter %r" % k)
        setattr(p, k, v)
    return p


def nominal(dur_ms: float) -> np.ndarray:
    out = np.zeros(P, np.float32)
    lib.opmm_nominal(ctypes.c_float(dur_ms), out.ctypes.data_as(ctypes.c_void_p))
    return out


def tile_names():
    return [lib.opmm_tile_name(i).decode() for i in range(lib.opmm_tile_count())]


def _ptr(t):
    if t is None:
        return None
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous(), "need a contiguous CUDA tensor"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def saccade_records(T, C, amp, dir_deg, dur_ms, seed, n_cand=None, pos_offset=None) -> np.ndarray:
    """Host opmm_saccade records; offsets default to back-to-back [T][C] traces."""
    T = np.asarray(T, np.int64).reshape(-1)
    S = T.shape[0]
    rec = np.zeros(S, SACCADE_DTYPE)
    Cs = np.broadcast_to(np.asarray(C, np.int64), (S,))
    if pos_offset is None:
        pos_offset = np.concatenate([[0], np.cumsum(T * Cs)[:-1]]) if S else np.zeros(0, np.int64)
    rec["pos_offset"] = pos_offset
    rec["T"] = T
    rec["C"] = Cs
    rec["amp_deg"] = amp
    rec["dir_deg"] = dir_deg
    rec["dur_ms"] = dur_ms
    rec["n_cand"] = 0 if n_cand is None else n_cand
    rec["seed"] = np.asarray(seed, np.uint64)
    return rec


class Context:
    """One libopmm context on one device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        rc = lib.opmm_create(ctypes.byref(h), int(device))
        if rc != OK:
            raise OpmmError(rc, "opmm_create(device=%d) failed" % device)
        self._h = h

    def close(self):
        if self._h:
            lib.opmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            raise OpmmError(rc, lib.opmm_last_error(self._h).decode())

    # -- calls -------------------------------------------------------------------------------
    def set_wait_limit(self, polls):
        self._check(lib.opmm_set_wait_limit(self._h, int(polls)))

    def kernel_timing(self, on):
        """Switch per-kernel event timing of directly queued fits on or off."""
        self._check(lib.opmm_kernel_timing_enable(self._h, 1 if on else 0))

    def kernel_times(self, kernel):
        """(total ms, launches) of `kernel` (KERNEL_*) since its last read; waits for them."""
        ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
        self._check(lib.opmm_kernel_timing_read(self._h, int(kernel), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def sync(self, stream=None):
        """Synchronise the stream; raises OpmmError(EDEVICE) if a persistent launch gave up a wait."""
        self._check(lib.opmm_sync(self._h, _stream(stream)))

    def candidates(self, seed, rnd, idx0, n, c, w, lo, hi, out, stream=None):
        arr = [np.ascontiguousarray(a, np.float32) for a in (c, w, lo, hi)]
        ps = [a.ctypes.data_as(ctypes.c_void_p) for a in arr]
        self._check(lib.opmm_candidates(self._h, ctypes.c_uint64(int(seed)), int(rnd), int(idx0), int(n),
                                        *ps, _ptr(out), _stream(stream)))

    def simulate(self, opc, amp, T, traj_out, dt_ms=1.0, stream=None):
        n = opc.shape[0]
        self._check(lib.opmm_simulate(self._h, _ptr(opc), _ptr(amp), n, int(T), ctypes.c_float(dt_ms),
                                      _ptr(traj_out), _stream(stream)))

    def score(self, opc, pos, sac_rec, rmse_out, dt_ms=1.0, stream=None, screen=False):
        """RMSE of candidates against one saccade; screen=True: with the screening pass's FP32 recurrence."""
        rec = np.ascontiguousarray(sac_rec, SACCADE_DTYPE).reshape(1)
        fn = lib.opmm_score_screen if screen else lib.opmm_score
        self._check(fn(self._h, _ptr(opc), opc.shape[0], _ptr(pos), pos.numel(),
                       rec.ctypes.data_as(ctypes.c_void_p), ctypes.c_float(dt_ms), _ptr(rmse_out), _stream(stream)))

    def fit(self, pos, recs, params: FitParams, opc_out, rmse_out, mae_out=None, status_out=None,
            round_keys=None, seed_opc=None, stream=None):
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        self._check(lib.opmm_fit(self._h, _ptr(pos), pos.numel(), recs.ctypes.data_as(ctypes.c_void_p),
                                 recs.shape[0], ctypes.byref(params), _ptr(seed_opc), _ptr(opc_out),
                                 _ptr(rmse_out), _ptr(mae_out), _ptr(status_out), _ptr(round_keys),
                                 _stream(stream)))

    def fit_noalloc(self, pos, recs, params: FitParams, opc_out, rmse_out, mae_out=None, status_out=None,
                    round_keys=None, seed_opc=None, stream=None):
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        self._check(lib.opmm_fit_noalloc(self._h, _ptr(pos), pos.numel(), recs.ctypes.data_as(ctypes.c_void_p),
                                         recs.shape[0], ctypes.byref(params), _ptr(seed_opc), _ptr(opc_out),
                                         _ptr(rmse_out), _ptr(mae_out), _ptr(status_out), _ptr(round_keys),
                                         _stream(stream)))

    def fit_nm(self, pos, recs, params: NmParams, opc_out, rmse_out, iters_out=None, decisions_out=None,
               status_out=None, seed_opc=None, stream=None):
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        self._check(lib.opmm_fit_nm(self._h, _ptr(pos), pos.numel(), recs.ctypes.data_as(ctypes.c_void_p),
                                    recs.shape[0], ctypes.byref(params), _ptr(seed_opc), _ptr(opc_out),
                                    _ptr(rmse_out), _ptr(iters_out), _ptr(decisions_out), _ptr(status_out),
                                    _stream(stream)))

    def sensitivity(self, recs, opc, theta_out, jac_out, dt_ms=1.0, stream=None):
        """Trajectories (FP64 [sum T]) and d theta / d p (FP64 [sum T][18]) at opc (device [S][18])."""
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        self._check(lib.opmm_sensitivity(self._h, recs.ctypes.data_as(ctypes.c_void_p), recs.shape[0], _ptr(opc),
                                         ctypes.c_float(dt_ms), _ptr(theta_out), _ptr(jac_out), _stream(stream)))

    def polish(self, pos, recs, params: PolishParams, opc_inout, rmse_out, mae_out=None, iters_out=None,
               decisions_out=None, model=18, stream=None):
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        self._check(lib.opmm_polish(self._h, _ptr(pos), pos.numel(), recs.ctypes.data_as(ctypes.c_void_p),
                                    recs.shape[0], ctypes.byref(params), int(model), _ptr(opc_inout),
                                    _ptr(rmse_out), _ptr(mae_out), _ptr(iters_out), _ptr(decisions_out),
                                    _stream(stream)))

    def ivt_extract(self, gaze, pos_out, dt_ms=1.0, vel_thresh=30.0, min_dur=6.0, min_amp=0.0, max_T=MAX_T,
                    seed_base=0, max_out=4096, stream=None):
        """Saccades of a gaze stream (device [N][2]) -> (records, first-sample indices); traces in pos_out."""
        recs = np.zeros(max_out, SACCADE_DTYPE)
        src = np.zeros(max_out, np.int64)
        n = ctypes.c_int32()
        self._check(lib.opmm_ivt_extract(self._h, _ptr(gaze), gaze.shape[0], ctypes.c_float(dt_ms),
                                         ctypes.c_float(vel_thresh), ctypes.c_float(min_dur),
                                         ctypes.c_float(min_amp), int(max_T), ctypes.c_uint64(seed_base),
                                         int(max_out), recs.ctypes.data_as(ctypes.c_void_p), _ptr(pos_out),
                                         pos_out.numel(), src.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n),
                                         _stream(stream)))
        return recs[:n.value], src[:n.value]

    def autotune(self, pos, recs, params: FitParams, stream=None) -> int:
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        t = ctypes.c_int32(-1)
        self._check(lib.opmm_autotune(self._h, _ptr(pos), pos.numel(), recs.ctypes.data_as(ctypes.c_void_p),
                                      recs.shape[0], ctypes.byref(params), ctypes.byref(t), _stream(stream)))
        return t.value

    def tune_cache_lookup(self, recs, params: FitParams) -> int:
        """The shape the autotuner cache holds for this batch, or -1."""
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        t = ctypes.c_int32(-1)
        self._check(lib.opmm_tune_cache_lookup(self._h, recs.ctypes.data_as(ctypes.c_void_p), recs.shape[0],
                                               ctypes.byref(params), ctypes.byref(t)))
        return t.value

    def tune_cache_save(self, path):
        self._check(lib.opmm_tune_cache_save(self._h, os.fsencode(path)))

    def tune_cache_load(self, path):
        self._check(lib.opmm_tune_cache_load(self._h, os.fsencode(path)))

    def plan(self, pos, recs, params: FitParams, opc_out, rmse_out, mae_out=None, status_out=None,
             round_keys=None, seed_opc=None, stream=None) -> "Plan":
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        h = ctypes.c_void_p()
        self._check(lib.opmm_fit_plan_create(self._h, _ptr(pos), pos.numel(),
                                             recs.ctypes.data_as(ctypes.c_void_p), recs.shape[0],
                                             ctypes.byref(params), _ptr(seed_opc), _ptr(opc_out),
                                             _ptr(rmse_out), _ptr(mae_out), _ptr(status_out),
                                             _ptr(round_keys), _stream(stream), ctypes.byref(h)))
        return Plan(self, h)


class Surrogate:
    """The learned seed (include/opmm.h, 'Learned seed')."""

    WIDTHS = (256, 512, 512, 256, 18)

    def __init__(self, ctx: Context, init_seed: int = 1):
        h = ctypes.c_void_p()
        ctx._check(lib.opmm_surrogate_create(ctx._h, ctypes.c_uint64(init_seed), ctypes.byref(h)))
        self._ctx, self._h = ctx, h

    def close(self):
        if self._h:
            lib.opmm_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def param_count() -> int:
        return int(lib.opmm_surrogate_param_count())

    def params(self, which=0) -> np.ndarray:
        out = np.zeros(self.param_count(), np.float32)
        self._ctx._check(lib.opmm_surrogate_get_params(self._h, which, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_params(self, w):
        w = np.ascontiguousarray(w, np.float32)
        assert w.shape == (self.param_count(),)
        self._ctx._check(lib.opmm_surrogate_set_params(self._h, w.ctypes.data_as(ctypes.c_void_p)))

    def forward(self, feat, out, stream=None):
        self._ctx._check(lib.opmm_surrogate_forward(self._h, _ptr(feat), feat.shape[0], _ptr(out), _stream(stream)))

    def backward(self, feat, target, stream=None, want_loss=True):
        """Forward + backward on one batch; returns the loss (which synchronises) or None."""
        loss = ctypes.c_float()
        self._ctx._check(lib.opmm_surrogate_backward(self._h, _ptr(feat), _ptr(target), feat.shape[0],
                                                     ctypes.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def adam_step(self, lr, stream=None):
        self._ctx._check(lib.opmm_surrogate_adam_step(self._h, ctypes.c_float(lr), _stream(stream)))

    def generate(self, data_seed, step, feat_out, target_out, spread=0.3, sigma_max=0.1, stream=None):
        self._ctx._check(lib.opmm_surrogate_generate(self._h, ctypes.c_uint64(data_seed), ctypes.c_uint64(step),
                                                     feat_out.shape[0], ctypes.c_float(spread),
                                                     ctypes.c_float(sigma_max), _ptr(feat_out), _ptr(target_out),
                                                     _stream(stream)))

    def train(self, data_seed, batch, n_steps, lr0=2e-3, lr_min=2e-5, spread=0.3, sigma_max=0.1,
              stream=None) -> np.ndarray:
        loss = np.zeros(max(n_steps, 1), np.float32)
        self._ctx._check(lib.opmm_surrogate_train(self._h, ctypes.c_uint64(data_seed), int(batch), int(n_steps),
                                                  ctypes.c_float(lr0), ctypes.c_float(lr_min),
                                                  ctypes.c_float(spread), ctypes.c_float(sigma_max),
                                                  loss.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return loss[:n_steps]

    def features(self, pos, recs, feat_out, dt_ms=1.0, stream=None):
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        self._ctx._check(lib.opmm_surrogate_features(self._h, _ptr(pos), pos.numel(),
                                                     recs.ctypes.data_as(ctypes.c_void_p), recs.shape[0],
                                                     ctypes.c_float(dt_ms), _ptr(feat_out), _stream(stream)))

    def predict(self, pos, recs, opc_out, dt_ms=1.0, box_frac=0.25, stream=None):
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        self._ctx._check(lib.opmm_surrogate_predict(self._h, _ptr(pos), pos.numel(),
                                                    recs.ctypes.data_as(ctypes.c_void_p), recs.shape[0],
                                                    ctypes.c_float(dt_ms), ctypes.c_float(box_frac),
                                                    _ptr(opc_out), _stream(stream)))

    def fit(self, pos, recs, seeded: FitParams, plain: FitParams, fallback_rmse, opc_out, rmse_out, status_out,
            mae_out=None, stream=None) -> int:
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        nf = ctypes.c_int32(0)
        self._ctx._check(lib.opmm_fit_learned(self._h, _ptr(pos), pos.numel(), recs.ctypes.data_as(ctypes.c_void_p),
                                              recs.shape[0], ctypes.byref(seeded), ctypes.byref(plain),
                                              ctypes.c_float(fallback_rmse), _ptr(opc_out), _ptr(rmse_out),
                                              _ptr(mae_out), _ptr(status_out), ctypes.byref(nf), _stream(stream)))
        return nf.value

    def save(self, path):
        self._ctx._check(lib.opmm_surrogate_save(self._h, os.fsencode(path)))

    def load(self, path):
        self._ctx._check(lib.opmm_surrogate_load(self._h, os.fsencode(path)))


def serve_params(**kw) -> ServeParams:
    p = ServeParams()
    lib.opmm_serve_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k in ("plain", "seeded") and isinstance(v, dict):
            for kk, vv in v.items():
                setattr(getattr(p, k), kk, vv)
        else:
            setattr(p, k, v)
    return p


class Server:
    """Continuous-batching estimation server (include/opmm.h, 'Continuous-batching server')."""

    def __init__(self, ctx: Context, params: ServeParams, surrogate: "Surrogate" = None):
        h = ctypes.c_void_p()
        ctx._check(lib.opmm_server_create(ctx._h, surrogate._h if surrogate else None, ctypes.byref(params),
                                          ctypes.byref(h)))
        self._ctx, self._h, self._sg = ctx, h, surrogate

    def close(self):
        if self._h:
            lib.opmm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def now() -> float:
        return lib.opmm_server_now()

    @property
    def slots(self) -> int:
        return lib.opmm_server_slots(self._h)

    def submit(self, trace, rec, t_arrival=None) -> int:
        trace = np.ascontiguousarray(trace, np.float32)
        rec = np.ascontiguousarray(rec, SACCADE_DTYPE).reshape(1)
        rid = ctypes.c_int64()
        self._ctx._check(lib.opmm_server_submit(self._h, trace.ctypes.data_as(ctypes.c_void_p),
                                                rec.ctypes.data_as(ctypes.c_void_p),
                                                self.now() if t_arrival is None else float(t_arrival),
                                                ctypes.byref(rid)))
        return rid.value

    def submit_many(self, host_pos, recs, t_arrival) -> np.ndarray:
        """host_pos: packed float32 traces (numpy), recs: records locating them, t_arrival: [n] seconds."""
        host_pos = np.ascontiguousarray(host_pos, np.float32)
        recs = np.ascontiguousarray(recs, SACCADE_DTYPE)
        ta = np.ascontiguousarray(t_arrival, np.float64)
        ids = np.zeros(recs.shape[0], np.int64)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._ctx._check(lib.opmm_server_submit_many(self._h, p(host_pos), host_pos.size, p(recs), recs.shape[0],
                                                     p(ta), p(ids)))
        return ids

    def step(self) -> int:
        n = ctypes.c_int32()
        self._ctx._check(lib.opmm_server_step(self._h, ctypes.byref(n)))
        return n.value

    _POLL_CHUNK = 4096

    def poll(self, max_n=1 << 30) -> dict:
        """Every finished result (up to max_n), oldest first.  Results are read in chunks through
        buffers kept on the server object, so a poll in a serving loop allocates only its output."""
        if not hasattr(self, "_pbuf"):
            c = self._POLL_CHUNK
            self._pbuf = (np.empty(c, np.int64), np.empty((c, P), np.float32), np.empty(c, np.float32),
                          np.empty(c, np.float32), np.empty(c, np.int32), np.empty(c), np.empty(c))
        ids, opc, rm, ma, st, ta, td = self._pbuf
        n = ctypes.c_int64()
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        parts, got = [], 0
        while got < max_n:
            want = int(min(self._POLL_CHUNK, max_n - got))
            self._ctx._check(lib.opmm_server_poll(self._h, want, p(ids), p(opc), p(rm), p(ma), p(st), p(ta), p(td),
                                                  ctypes.byref(n)))
            k = n.value
            parts.append([a[:k].copy() for a in (ids, opc, rm, ma, st, ta, td)])
            got += k
            if k < want:
                break
        cols = [np.concatenate([q[i] for q in parts]) for i in range(7)]
        return dict(id=cols[0], opc=cols[1], rmse=cols[2], mae=cols[3], status=cols[4], t_arrival=cols[5],
                    t_done=cols[6])

    def stats(self) -> dict:
        out = np.zeros(7, np.int64)
        self._ctx._check(lib.opmm_server_stats(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return dict(zip(("pending", "busy", "admitted", "completed", "fallbacks", "steps", "slots"), map(int, out)))


class Plan:
    """A fit captured in a HIP graph; launch() replays it."""

    def __init__(self, ctx: Context, h):
        self._ctx, self._h = ctx, h

    def launch(self, stream=None):
        rc = lib.opmm_plan_launch(self._h, _stream(stream))
        if rc != OK:
            raise OpmmError(rc, lib.opmm_last_error(self._ctx._h).decode())

    def close(self):
        if self._h:
            lib.opmm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack_traces(traces):
    """List of [T_i][C] float arrays -> one packed float32 array (the pos buffer)."""
    if not traces:
        return np.zeros(0, np.float32)
    return np.concatenate([np.asarray(t, np.float32).reshape(-1) for t in traces])
