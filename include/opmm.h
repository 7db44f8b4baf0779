/*
 * opmm.h -- C ABI of the MI355X (gfx950) OPMM estimation library, libopmm.so.
 *
 * The library estimates oculomotor plant characteristics (OPCs) from recorded
 * saccades as described in "Parallel Oculomotor Plant Mathematical Model for
 * Large Scale Eye Movement Simulation" (Karpov, Liberman, Lohr, Komogortsev,
 * arXiv 2007.09884): a saccade trajectory goes in, an 18-parameter OPC vector
 * comes out (Section 2, problem statement; Algorithm 1 input/output;
 * Section 3.4 output = OPC vector plus optimisation error).  The plant is the
 * 18-parameter model of Section 2.2.1 (Table 1 lists the parameters), driven
 * by the pulse-step control of Section 2.1.
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers unless marked "host".  The caller
 *     owns them; they must stay valid until the work queued on `stream` has
 *     completed.  The library keeps no caller pointer past that point (the
 *     plan calls below are the one exception and say so).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is queued on it; calls return once it is queued.
 *   - Return value: OPMM_OK or a negative OPMM_E* code; no exception crosses
 *     the ABI.  opmm_last_error() gives the text of the last failure on that
 *     context.  Argument errors are detected on the host before anything is
 *     queued.
 *   - OPC vectors are FP32 [18] in Table 1 order:
 *       0 K_SE_AG   1 K_SE_ANT  2 K_LT_AG   3 K_LT_ANT  (g/deg)
 *       4 B_AG      5 B_ANT     6 B_P                   (g s/deg)
 *       7 N_C_AG    8 N_C_ANT                            (g/deg)
 *       9 J                                              (g s^2/deg)
 *      10 tau_AC_AG 11 tau_AC_ANT 12 tau_DE_AG 13 tau_DE_ANT (ms)
 *      14 N_C_FIX  15 N_SAC_AG  16 N_SAC_ANT             (g)
 *      17 PW                                             (ms)
 *   - A context is bound to one device and is not thread-safe; calls on one
 *     context must not overlap.
 *   - Streams: a context, a surrogate and a plan each reuse device scratch
 *     from call to call.  Calls on one object may use different streams: the
 *     library orders them itself, so each call's device work starts after the
 *     previous call's (the first call on a second stream waits on the host
 *     for the device to drain; later calls wait on an event, on the device).
 *     Calls that all use one stream add nothing to it.  A call queued under
 *     stream capture is left out of this ordering; inside a graph the caller
 *     orders the work.  opmm_fit_noalloc's scratch is one per device, shared
 *     by every context (see there).
 */
#ifndef OPMM_H
#define OPMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OPMM_P 18          /* OPC vector length (Table 1)                */
#define OPMM_MAX_T 2048    /* longest trace, samples                      */

enum {
    OPMM_OK = 0,
    OPMM_EINVAL = -1,      /* bad argument; nothing was queued            */
    OPMM_ENOMEM = -2,      /* device or pinned-host allocation failed     */
    OPMM_EDEVICE = -3,     /* HIP runtime error                           */
    OPMM_ENOTREADY = -4    /* object not initialised (e.g. no surrogate)  */
};

/* Per-saccade status bits written by opmm_fit. */
enum {
    OPMM_ST_OK = 0,
    OPMM_ST_NONFINITE_INPUT = 1,    /* trace holds NaN/Inf: not fitted, outputs NaN */
    OPMM_ST_NO_FINITE_CANDIDATE = 2,/* some round had no candidate with finite cost */
    OPMM_ST_SEEDED = 4,             /* search started from a supplied/learned seed  */
    OPMM_ST_FALLBACK = 8,           /* seeded result rejected; plain search used    */
    OPMM_ST_WAIT_TIMEOUT = 16,      /* persistent launch: a tile gave up waiting for
                                       its round (opmm_set_wait_limit); that tile
                                       was not searched, the result is no estimate */
    OPMM_ST_DEADLINE = 32           /* Nelder-Mead: the time bound ended the task
                                       before its tolerances held (best vertex so far) */
};

/* Search kernels that opmm_kernel_timing_read reports on. */
enum {
    OPMM_KERNEL_ROUND = 0,       /* one FP64 round of every tile (per-round mode)       */
    OPMM_KERNEL_SCREEN = 1,      /* FP32 pass of a screened round                       */
    OPMM_KERNEL_VERIFY = 2,      /* FP64 re-simulation of a screened round's survivors
                                    (the FP64 anchor launch before it is not timed)     */
    OPMM_KERNEL_PERSISTENT = 3,  /* the work-queue launch of a persistent fit           */
    OPMM_KERNEL_KINDS = 4
};

typedef struct opmm_ctx opmm_ctx;

/* One recorded saccade (Section 3.1: extracted saccades are the input).
 * Host-side record; its trace lives in a packed device buffer of FP32
 * positions (deg), [T][C] row-major, starting at element pos_offset.
 * Time 0 (sample 0) is the pulse onset.  The plant is one-dimensional
 * (Section 2.2) and moves along direction dir_deg: with C = 2 the predicted
 * trace is theta*(cos dir, sin dir); with C = 1 the single channel is the
 * horizontal one and dir_deg must be 0 or 180. */
typedef struct {
    int64_t pos_offset;  /* first element of this trace in `pos`             */
    int32_t T;           /* samples, 1..OPMM_MAX_T                           */
    int32_t C;           /* channels: 1 (H) or 2 (H, V)                      */
    float amp_deg;       /* amplitude A >= 0: the post-saccadic fixation     */
    float dir_deg;       /* direction of the movement                        */
    float dur_ms;        /* duration D > 6: nominal PW = D - 6 (Table 1)     */
    int32_t n_cand;      /* candidates per round; 0 = opmm_fit_params.n_cand */
    uint64_t seed;       /* key of the candidate stream: results depend only
                            on (seed, trace, params), never on batch layout  */
} opmm_saccade;

enum { OPMM_FIT_ROUNDS = 0, OPMM_FIT_PERSISTENT = 1 };

/* Box search parameters.  Round r draws n_cand candidates uniformly in
 * centre^r +/- w^r (candidate 0 = centre^r), clamped to the search box
 * nominal +/- box_frac*nominal; the argmin (lowest RMSE, ties to the lowest
 * index) becomes centre^{r+1} and w^{r+1} = shrink*w^r.  Round 0 is centred
 * on the nominal OPC (Section 3.2: initialised to literature defaults) or on
 * a supplied seed, with w^0 = w_init_frac*box_frac*nominal. */
typedef struct {
    int32_t n_cand;      /* default candidates per round, >= 1               */
    int32_t n_rounds;    /* rounds R, 1..4096                                */
    float box_frac;      /* search box half-width / nominal, (0, 1)  [0.25]  */
    float w_init_frac;   /* round-0 half-width / box half-width, [0, 1] [1]  */
    float shrink;        /* half-width factor per round, (0, 1]      [0.5]   */
    float dt_ms;         /* sample period, (0, 1]                    [1.0]   */
    int32_t mode;        /* OPMM_FIT_ROUNDS: one launch per round;
                            OPMM_FIT_PERSISTENT: one work-queue launch for
                            every round and saccade (uneven batches)         */
    int32_t tile;        /* kernel shape index; -1 = autotuned/default, and
                            the 512-candidate tile for a launch with fewer
                            tiles than the device has CUs (same results,
                            each block finishes sooner)                      */
    int32_t model;       /* 18: the 18-parameter OPMM (Section 2.2.1);
                            9: the 9-parameter OPMM (Section 2.2.2, Table 2):
                            one K_SE and one K_LT for both muscles (the
                            stream's K_SE_ANT := K_SE_AG, K_LT_ANT := K_LT_AG)
                            and the neural parameters (tau_AC/DE, N_SAC, PW)
                            held at nominal (half-width 0)                   */
    int32_t screen_rounds; /* rounds 0..screen_rounds-1 are screened: every
                            candidate is simulated with an FP32 recurrence;
                            the FP32 best b is simulated again in FP64, and
                            only the candidates whose FP32 RMSE is at most
                            RMSE64(b) + screen_tol / 2 are simulated again
                            in FP64, which decides the argmin.  The winner
                            is the FP64 argmin whenever the FP32 RMSE
                            errors stay below screen_tol / 2 (measured:
                            below 8.6e-6 deg; opmm_score_screen measures
                            them).  0 = every round in FP64 only.
                            Per-round mode only; 0..n_rounds           [0]   */
    float screen_tol;    /* deg of RMSE, > 0                         [5e-5]  */
} opmm_fit_params;

/* Defaults: n_cand 4096, n_rounds 1, box 0.25, w_init 1, shrink 0.5, dt 1 ms,
 * model 18, no screening (tolerance 5e-5 deg when enabled). */
void opmm_fit_params_default(opmm_fit_params* p);

/* Nominal OPC for a saccade of duration dur_ms (Table 1; PW = D - 6 ms).
 * host out[18]. */
void opmm_nominal(float dur_ms, float* out);

/* Context: binds a device, owns the device scratch (per-saccade search state,
 * projected traces, round keys) and the autotuner cache.  Scratch grows on
 * demand and is freed by opmm_destroy. */
int opmm_create(opmm_ctx** out, int device);
int opmm_destroy(opmm_ctx* ctx);
const char* opmm_last_error(const opmm_ctx* ctx);

/* The persistent launch (OPMM_FIT_PERSISTENT) has blocks wait on the device
 * for the previous round of their saccade (Algorithm 1 runs the rounds of a
 * task in order).  The wait is bounded by `polls` polls (default 2^26, several
 * seconds); a block that gives up leaves its tile unsearched, sets
 * OPMM_ST_WAIT_TIMEOUT on that saccade and is counted in the context's
 * report, and the launch still runs to its end.  0 makes every such wait give
 * up at once (to exercise the report).  Applies to fits queued and plans
 * created after the call. */
int opmm_set_wait_limit(opmm_ctx* ctx, uint32_t polls);
/* Kernel timing, a measurement aid with no counterpart in the paper.  With
 * timing on, each fit queued directly on a stream (opmm_fit, opmm_fit_learned,
 * opmm_fit_noalloc, and the one uncaptured run opmm_fit_plan_create makes
 * before it captures; not a plan's graph launches, nothing under stream
 * capture) records a HIP event pair on its stream around every launch of a
 * search kernel (OPMM_KERNEL_*); the
 * events come from a pool of 1024 pairs made when timing is switched on
 * (host-side event objects, no device memory), and launches beyond that many
 * between two reads are not timed.  Event timing adds a few microseconds per
 * launch to the stream.  Off by default; `on` = 0 switches it off and keeps
 * the pool until the context is destroyed. */
int opmm_kernel_timing_enable(opmm_ctx* ctx, int32_t on);
/* Wait for the recorded launches of `kernel` (OPMM_KERNEL_*), then return
 * their summed duration in ms and their count since the last read of that
 * kernel, and clear both.  OPMM_EINVAL for a null handle or output or an
 * unknown kernel. */
int opmm_kernel_timing_read(opmm_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches);

/* Synchronise `stream`, then read and clear the context's report: returns
 * OPMM_EDEVICE (with the count in opmm_last_error) if any persistent launch
 * of this context that has completed gave up a wait since the last call,
 * else OPMM_OK. */
int opmm_sync(opmm_ctx* ctx, void* stream);

/* Candidate vectors of the search stream (for replay and for callers that
 * score their own candidate sets).  Writes out[n][18] for candidate indices
 * idx0 .. idx0+n-1 of round `round` of the stream keyed by `seed`, drawn
 * around centre c with half-width w and clamped to [lo, hi] (all host [18]).
 * Rule: SplitMix64 output 1 + (round<<36 | idx<<4 | k), k = 0..8, gives two
 * 24-bit uniforms u (top 24 bits -> parameter 2k, next 24 -> 2k+1);
 * s = u/2^23 - 1; p = clamp(fmaf(w, s, c), lo, hi).  Index 0 is c itself. */
int opmm_candidates(opmm_ctx* ctx, uint64_t seed, uint32_t round, uint32_t idx0, int64_t n,
                    const float* c, const float* w, const float* lo, const float* hi,
                    float* out, void* stream);

/* Simulate the plant (Sections 2.1-2.2.1) for n OPC vectors opc[n][18], each
 * with its own amplitude amp[n] (deg): the eye rests at 0, the pulse acts on
 * [0, PW), the step holds amp afterwards.  traj_out[n][T] = theta at t_k =
 * k*dt_ms (deg).  FP32; within 1e-4 deg of the FP64 solution for OPCs within
 * +/-30% of nominal.  T in 1..OPMM_MAX_T. */
int opmm_simulate(opmm_ctx* ctx, const float* opc, const float* amp, int64_t n, int32_t T,
                  float dt_ms, float* traj_out, void* stream);

/* Score n candidate OPC vectors opc[n][18] against one saccade: rmse_out[n] =
 * sqrt(sum_k sum_c (pos - pred)^2 / (C*T)), the fit criterion (NaN -> +Inf).
 * pos is the packed trace buffer of pos_len elements; sac (host) locates the
 * trace.  The optimisation error of Section 3.4, recomputed per candidate. */
int opmm_score(opmm_ctx* ctx, const float* opc, int64_t n, const float* pos, int64_t pos_len,
               const opmm_saccade* sac, float dt_ms, float* rmse_out, void* stream);
/* opmm_score with the FP32 recurrence of screened rounds (opmm_fit_params.
 * screen_rounds): for each candidate the very operations of the FP32 pass,
 * so max |opmm_score_screen - opmm_score| over a caller's candidates is the
 * screening error eps on that data, which must stay below screen_tol / 2 for
 * a screened fit to return the FP64 fit (the argmin argument is the FP64
 * argmin's FP32 RMSE <= FP32 best + 2 eps).  A measurement aid; arguments,
 * layout and errors as opmm_score. */
int opmm_score_screen(opmm_ctx* ctx, const float* opc, int64_t n, const float* pos, int64_t pos_len,
                      const opmm_saccade* sac, float dt_ms, float* rmse_out, void* stream);

/* Estimate the OPC vector of each of S saccades (Algorithm 1: one task per
 * saccade, all on the device; Section 3.3: the data stay on the GPU).
 *   pos, pos_len   packed traces (device), see opmm_saccade
 *   sacs           host [S]
 *   seed_opc       NULL, or device [S][18] round-0 centres (clamped into the
 *                  box; a NaN component keeps the nominal centre; status
 *                  gets OPMM_ST_SEEDED)
 *   opc_out        device [S][18]  fitted OPC (the final argmin)
 *   rmse_out       device [S]      its RMSE over both channels (deg)
 *   mae_out        NULL or device [S]: its mean absolute difference (OptErr)
 *   status_out     NULL or device [S]: OPMM_ST_* bits
 *   round_keys     NULL or device [n_rounds][S]: per round the argmin key
 *                  (float bits of the winner's projected SSE << 32 | index)
 * Results are bit-identical between modes, kernel shapes and batch layouts. */
int opmm_fit(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs,
             int32_t S, const opmm_fit_params* params, const float* seed_opc, float* opc_out,
             float* rmse_out, float* mae_out, int32_t* status_out, uint64_t* round_keys,
             void* stream);

/* Allocation-free variant of opmm_fit, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and status words as opmm_fit, bit for
 * bit.  Its device scratch is one static array per device of
 * OPMM_NOALLOC_SCRATCH_BYTES, held until the process ends, and its host
 * staging a static buffer; the call makes no hipMalloc, hipFree or other
 * allocation.  Limits: S <= OPMM_NOALLOC_MAX_S and a scratch layout within
 * OPMM_NOALLOC_SCRATCH_BYTES (per saccade 80 B record, 8 B order, 8 B energy,
 * 288 B box, 4 B status, 8 B counters and, without round_keys, 8 B per round;
 * 4 B per trace sample; each part 256-byte aligned), else OPMM_EINVAL.  Every
 * call on a device shares that device's array and keeps the last call's
 * contents (each call rewrites every part before reading it).  Calls through
 * one context are ordered across streams as every call on a context is;
 * calls through different contexts or threads that overlap on one device
 * race, so the caller must order them.  Like opmm_fit it uploads the records
 * synchronously and queues the rest on `stream`. */
#define OPMM_NOALLOC_MAX_S 4096
#define OPMM_NOALLOC_SCRATCH_BYTES (8u << 20)
int opmm_fit_noalloc(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs,
                     int32_t S, const opmm_fit_params* params, const float* seed_opc, float* opc_out,
                     float* rmse_out, float* mae_out, int32_t* status_out, uint64_t* round_keys,
                     void* stream);

/* A fit captured once into a HIP graph and replayed: the same work as
 * opmm_fit with the same arguments, bound to these buffers.  Creation runs
 * the fit once (synchronously) and then captures it; opmm_plan_launch replays
 * the whole fit as one graph launch.  The plan owns its own device scratch
 * and keeps the caller's device pointers (not the host records) until
 * opmm_plan_destroy; replays must not overlap each other. */
typedef struct opmm_plan opmm_plan;
int opmm_fit_plan_create(opmm_ctx* ctx, const float* pos, int64_t pos_len,
                         const opmm_saccade* sacs, int32_t S, const opmm_fit_params* params,
                         const float* seed_opc, float* opc_out, float* rmse_out, float* mae_out,
                         int32_t* status_out, uint64_t* round_keys, void* stream,
                         opmm_plan** out);
int opmm_plan_launch(opmm_plan* plan, void* stream);
int opmm_plan_destroy(opmm_plan* plan);

/* Autotuner: time every kernel shape on a representative sample of this
 * batch (at most 256 saccades, up to 4 rounds, the caller's mode) and keep
 * the fastest for later calls on this context with tile = -1.
 * Writes the chosen shape index to *tile_out (host, nullable). */
int opmm_autotune(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs,
                  int32_t S, const opmm_fit_params* params, int32_t* tile_out, void* stream);
/* Autotuner cache.  Each opmm_autotune also files its pick under the batch's
 * key: launch mode, model, the longest trace and the batch size each rounded
 * up to a power of two, and the largest candidate count.  A later fit, plan
 * or learned fit with tile = -1 whose batch has a filed key runs that shape;
 * other batches keep the context's last pick, or the library default.
 *   opmm_tune_cache_lookup: the filed shape of a batch in *tile_out (host), or
 *     -1 if none.  Host only.
 *   opmm_tune_cache_save: writes the context's entries to a text file, one
 *     line each: device architecture name, the key, shape name, measured ms.
 *   opmm_tune_cache_load: adds the entries of such a file that were written
 *     for this device's architecture (other lines, and shapes this build
 *     does not have, are skipped; a filed key is replaced).  Nothing is added
 *     if any line is malformed.
 * Errors: OPMM_EINVAL for a NULL argument, a file that cannot be opened or
 * written, or a malformed line (opmm_last_error names it). */
int opmm_tune_cache_lookup(opmm_ctx* ctx, const opmm_saccade* sacs, int32_t S,
                           const opmm_fit_params* params, int32_t* tile_out);
int opmm_tune_cache_save(opmm_ctx* ctx, const char* path);
int opmm_tune_cache_load(opmm_ctx* ctx, const char* path);
/* Number of kernel shapes, a description of shape i (host string), and the
 * shape used for tile = -1 on a context that has not been autotuned (the
 * fastest per-round shape of a sweep on the full-estimation workload). */
int opmm_tile_count(void);
const char* opmm_tile_name(int i);
int opmm_tile_default(void);


/* ------------------------------------------------------------------------
 * Learned seed: a small MLP (256-512-512-256-18, ReLU, BF16 weights and
 * activations, FP32 accumulate) that maps a saccade trace to an initial OPC
 * estimate, trained on saccades the plant simulator itself generates; the
 * box search refines from it and stays both its fallback and the judge of
 * its error.  Not in the paper: the learned counterpart of its literature-
 * default initialisation (Section 3.2) and of its call for faster estimation
 * toward real time (Section 5).
 *   input  = the trace projected on the movement direction, resampled to
 *            128 points over its own duration, as (position/16 deg,
 *            velocity*4 ms/deg) pairs: [256] BF16 (raw uint16 bit patterns)
 *   output = z = (p / p_nominal - 1) / 0.3 per Table 1 component [18] FP32
 * Parameters are one FP32 vector of opmm_surrogate_param_count() values:
 * W0 [256][512], b0, W1 [512][512], b1, W2 [512][256], b2, W3 [256][18], b3.
 * ------------------------------------------------------------------------ */
typedef struct opmm_surrogate opmm_surrogate;

/* He-uniform weights from the SplitMix64 stream keyed by init_seed. */
int opmm_surrogate_create(opmm_ctx* ctx, uint64_t init_seed, opmm_surrogate** out);
int opmm_surrogate_destroy(opmm_surrogate* sg);
int64_t opmm_surrogate_param_count(void);
/* which: 0 weights, 1 gradients of the last backward pass, 2/3 Adam moments;
 * host_out[param_count]; synchronises the device. */
int opmm_surrogate_get_params(opmm_surrogate* sg, int which, float* host_out);
int opmm_surrogate_set_params(opmm_surrogate* sg, const float* host_w);
/* out[B][18] = network(feat[B][256]) */
int opmm_surrogate_forward(opmm_surrogate* sg, const uint16_t* feat, int32_t B, float* out, void* stream);
/* forward + backward of the MSE loss mean((out - target)^2) over B x 18;
 * gradients are left in the object (get_params which = 1); *loss_out (host,
 * nullable) gets the loss, which synchronises the stream. */
int opmm_surrogate_backward(opmm_surrogate* sg, const uint16_t* feat, const float* target, int32_t B,
                            float* loss_out, void* stream);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) on the stored gradients. */
int opmm_surrogate_adam_step(opmm_surrogate* sg, float lr, void* stream);
/* Training data on the device: B saccades with OPC = nominal x U[1-spread,
 * 1+spread], amplitude U[2, 30] deg, duration 2.2 A + 21 ms, noise sigma
 * U[0, sigma_max] deg, keyed by (data_seed, step): feat_out[B][256],
 * target_out[B][18] (device). */
int opmm_surrogate_generate(opmm_surrogate* sg, uint64_t data_seed, uint64_t step, int32_t B, float spread,
                            float sigma_max, uint16_t* feat_out, float* target_out, void* stream);
/* n_steps of (generate batch -> forward -> backward -> Adam), learning rate
 * cosine-decayed from lr0 to lr_min over the call; loss_out (host, nullable)
 * [n_steps].  Synchronises the stream at the end. */
int opmm_surrogate_train(opmm_surrogate* sg, uint64_t data_seed, int32_t B, int32_t n_steps, float lr0,
                         float lr_min, float spread, float sigma_max, float* loss_out, void* stream);
/* Features of S recorded saccades (same layout rules as opmm_fit):
 * feat_out[S][256] (device). */
int opmm_surrogate_features(opmm_surrogate* sg, const float* pos, int64_t pos_len, const opmm_saccade* sacs,
                            int32_t S, float dt_ms, uint16_t* feat_out, void* stream);
/* Seeds for S saccades: opc_out[S][18] = nominal x (1 + 0.3 z), clamped to
 * nominal x [1 - box_frac, 1 + box_frac]; pass as seed_opc to opmm_fit. */
int opmm_surrogate_predict(opmm_surrogate* sg, const float* pos, int64_t pos_len, const opmm_saccade* sacs,
                           int32_t S, float dt_ms, float box_frac, float* opc_out, void* stream);
/* Learned-seed estimation: seeds from the network, then opmm_fit with
 * `seeded` (typically fewer candidates/rounds and w_init_frac < 1); every
 * saccade whose seeded RMSE exceeds fallback_rmse (e.g. 1.5 x the noise
 * floor) is re-fitted with `plain` from the nominal centre, and the lower-
 * RMSE result is kept (status gets OPMM_ST_FALLBACK).  status_out is
 * required.  *n_fallback (host, nullable) = number of re-fitted saccades.
 * Synchronises the stream once to read the seeded RMSEs. */
int opmm_fit_learned(opmm_surrogate* sg, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                     const opmm_fit_params* seeded, const opmm_fit_params* plain, float fallback_rmse,
                     float* opc_out, float* rmse_out, float* mae_out, int32_t* status_out, int32_t* n_fallback,
                     void* stream);
/* Checkpoint: FP32 weights and Adam state (binary, host file). */
int opmm_surrogate_save(opmm_surrogate* sg, const char* path);
int opmm_surrogate_load(opmm_surrogate* sg, const char* path);

/* ------------------------------------------------------------------------
 * Continuous-batching server: saccades streamed one by one are estimated
 * as they arrive (the real-time goal of Section 5: as fast as recording).
 * Each admitted request owns a device slot (trace, projection, search box,
 * status, round key stay resident in HBM); opmm_server_step advances every
 * occupied slot by one search round in one launch, whatever round each is
 * at, and admits waiting requests as slots free up.  While such a launch
 * would leave compute units idle (fewer candidate tiles than CUs), the step
 * runs further rounds for the slots still searching, up to rounds_per_step
 * launches: a light load then finishes a search in one step instead of one
 * step per round.  The slot count is the
 * HBM budget divided by one slot's footprint (capped by max_slots).  A
 * result depends only on its own request: the same alone and in the mix.
 * With a surrogate, requests start from the learned seed (`seeded`) and fall
 * back to `plain` when the seeded RMSE exceeds fallback_rmse (the lower-RMSE
 * result is kept, status gets OPMM_ST_FALLBACK); without, they run `plain`.
 * With polish_iter > 0, every finished search is polished (opmm_polish with
 * that many iterations, the RMSE objective, the searches' box and dt) before
 * the fallback rule and the result are taken; the polish runs on streams of
 * the server's own and its results are taken by a later step.
 * The server owns its streams; calls on one server must not overlap.
 * ------------------------------------------------------------------------ */
typedef struct opmm_server opmm_server;
typedef struct {
    int32_t max_slots;        /* upper bound on resident requests            */
    int32_t max_T;            /* longest trace accepted, <= OPMM_MAX_T       */
    size_t hbm_budget_bytes;  /* device memory the slots may use             */
    opmm_fit_params plain;    /* search from the nominal OPC (and fallback)  */
    opmm_fit_params seeded;   /* search from the learned seed                */
    float fallback_rmse;      /* deg; e.g. 1.5 x the noise floor             */
    int32_t polish_iter;      /* polish iterations per finished search, 0-100 */
    int32_t rounds_per_step;  /* most round launches in one step, 1-64     */
} opmm_serve_params;

/* Defaults: 4096 slots, max_T 160, 1 GiB; plain 4096 x 10, seeded 1024 x 3
 * with w_init_frac 0.25; fallback 0.075 deg; no polish; 16 rounds per step.  plain and seeded
 * must share dt_ms, box_frac and shrink. */
void opmm_serve_params_default(opmm_serve_params* p);
/* sg nullable (no learned seed).  The server keeps ctx and sg. */
int opmm_server_create(opmm_ctx* ctx, opmm_surrogate* sg, const opmm_serve_params* prm, opmm_server** out);
int opmm_server_destroy(opmm_server* sv);
int opmm_server_slots(const opmm_server* sv);
/* Seconds on the server's clock (steady); use it for arrival timestamps. */
double opmm_server_now(void);
/* Queue one request: host_trace [T][C] FP32 (copied), sac (host; pos_offset
 * ignored), t_arrival on opmm_server_now()'s clock.  *id_out = request id. */
int opmm_server_submit(opmm_server* sv, const float* host_trace, const opmm_saccade* sac, double t_arrival,
                       int64_t* id_out);
/* Queue n requests at once: traces in host_pos (pos_len floats) located by
 * sacs[i].pos_offset, arrival times t_arrival[n]; ids_out[n] nullable.  All
 * records are validated before any is queued. */
int opmm_server_submit_many(opmm_server* sv, const float* host_pos, int64_t pos_len, const opmm_saccade* sacs,
                            int32_t n, const double* t_arrival, int64_t* ids_out);
/* Admit, run one round over all occupied slots (more while the device would
 * sit idle, see above), harvest finished requests (synchronises the server
 * stream; polish batches still running are taken by a later step).  *n_done_out (nullable) = requests completed by this step. */
int opmm_server_step(opmm_server* sv, int32_t* n_done_out);
/* Pop up to max completed results (host arrays, each nullable except n_out):
 * ids[n], opc[n][18], rmse[n], mae[n], status[n], t_arrival[n], t_done[n]. */
int opmm_server_poll(opmm_server* sv, int64_t max, int64_t* ids, float* opc, float* rmse, float* mae,
                     int32_t* status, double* t_arrival, double* t_done, int64_t* n_out);
/* out[7] = pending, occupied slots, admitted, completed, fallbacks, steps, slots. */
int opmm_server_stats(const opmm_server* sv, int64_t* out);

/* ------------------------------------------------------------------------
 * The paper's estimator: parallel Nelder-Mead (Section 3.3, Algorithm 1) in
 * the variant of Lagarias et al. (reflection 1, expansion 2, contraction
 * 1/2, shrink 1/2), one task per saccade with all simplex transforms of an
 * iteration evaluated simultaneously and the simplex sorted (stable) every
 * iteration.  Coordinates are the OPC relative to the Table 1 nominal; the
 * initial simplex is x0 and x0 with one coordinate scaled by 1.05; the cost
 * (RMSE, as opmm_fit) is evaluated at the point clamped to nominal x
 * [1 - box_frac, 1 + box_frac] and rounded to FP32.  Exit when every vertex
 * is within tol_x of the best in every coordinate AND every value within
 * tol_f of the best (both, Section 3.3), or after max_iter iterations.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t max_iter;   /* iteration cap                    [500]  */
    float tol_x;        /* coordinate tolerance (relative)  [1e-4] */
    float tol_f;        /* value tolerance (deg RMSE)       [1e-6] */
    float box_frac;     /* evaluation clamp                 [0.25] */
    float dt_ms;        /* sample period                    [1.0]  */
    float max_ms;       /* time bound per task, ms of device wall clock
                           from the launch's start; 0 = none [0].  A task
                           still iterating then stops with its best vertex
                           and OPMM_ST_DEADLINE (Section 3.3 names a time
                           limit among the exit criteria)              */
    int32_t tasks_per_wave; /* 0 auto, 1 or 2 tasks per 64-lane wave   [0] */
} opmm_nm_params;
void opmm_nm_params_default(opmm_nm_params* p);
/* seed_opc: NULL (start at nominal) or device [S][18].  Outputs (device):
 * opc_out [S][18] best vertex, rmse_out [S] its cost, iters_out [S]
 * (nullable) iterations taken, decisions_out (nullable) [S][max_iter]:
 * per iteration 0 reflect, 1 expand, 2 outside contraction, 3 inside
 * contraction, 4 shrink; status_out (nullable) [S]. */
int opmm_fit_nm(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                const opmm_nm_params* prm, const float* seed_opc, float* opc_out, float* rmse_out, int32_t* iters_out,
                int8_t* decisions_out, int32_t* status_out, void* stream);

/* ------------------------------------------------------------------------
 * Forward sensitivities of the plant trajectory: d theta_k / d p_j for every
 * OPC component j (Table 1 order, per unit of the component), k < T, at the
 * given candidates.  The plant is linear and time-invariant on each piece of
 * the pulse-step control (Section 2.1), so the sensitivities are those of the
 * exact trajectory; PW's column is the effect of moving the pulse end.  This
 * is the gradient information that the gradient-based estimation the paper
 * proposes as future work (Section 5) needs.
 *   sacs      host [S]: only T, amp_deg and dur_ms are read
 *   opc       device [S][18] FP32
 *   theta_out device, FP64: saccade s's trajectory at [off_s, off_s + T_s),
 *             off_s = sum of T over the saccades before s
 *   jac_out   device, FP64 [sum T][18]: row off_s + k is d theta_k / d p
 * Synchronises the stream before returning (host records).  Errors:
 * OPMM_EINVAL (bad record, dt_ms outside (0, 1]); nothing is queued then. */
int opmm_sensitivity(opmm_ctx* ctx, const opmm_saccade* sacs, int32_t S, const float* opc, float dt_ms,
                     double* theta_out, double* jac_out, void* stream);

/* ------------------------------------------------------------------------
 * Gradient-based polish of fitted OPC vectors (the estimation alternative of
 * Section 5, applied after the box search): Levenberg-Marquardt with
 * Marquardt scaling in coordinates relative to the Table 1 nominal, Jacobian
 * from the forward sensitivities above taken on the search path's coarser
 * discretisation (it only shapes the step; the objective values that accept
 * or reject a step use the finer one of opmm_sensitivity).  Each iteration
 * solves the damped normal equations for 8 damping values at once
 * (lambda * 10^(m-4), m = 0..7) and takes the best trial point if it lowers the objective
 * (lambda becomes a tenth of the winner's), else raises lambda by 1e8.
 * Objective OPMM_OBJ_RMSE is the fit cost of Section 3.4; OPMM_OBJ_MAE is
 * the mean absolute difference reported as OptErr (Fig. 4), minimised by
 * iteratively reweighted least squares.  Points stay inside the search box
 * (nominal +/- box_frac, PW = D - 6 ms); components at a bound whose
 * gradient points outward are held.  With model 9 only the nine free
 * components move (K_SE and K_LT tied across muscles, the rest fixed at their
 * input values).  Stops when an accepted step gains less than tol_f times the
 * objective, when lambda exceeds 1e30, or after max_iter iterations. */
enum { OPMM_OBJ_RMSE = 0, OPMM_OBJ_MAE = 1 };
typedef struct {
    int32_t max_iter;   /* iteration cap                       [20]    */
    int32_t objective;  /* OPMM_OBJ_RMSE or OPMM_OBJ_MAE       [RMSE]  */
    float tol_f;        /* relative gain that ends the polish  [1e-10] */
    float lambda0;      /* initial damping                     [1e-3]  */
    float box_frac;     /* search box half-width / nominal     [0.25]  */
    float dt_ms;        /* sample period, (0, 1]               [1.0]   */
} opmm_polish_params;
void opmm_polish_params_default(opmm_polish_params* p);
/* pos, sacs as for opmm_fit (n_cand and seed unused).  opc_inout: device
 * [S][18], the start points in, the polished OPC out (never worse in the
 * objective than the start clamped to the box).  rmse_out (device [S]) and
 * mae_out (nullable) get both costs of the result; iters_out (nullable) the
 * iterations taken; decisions_out (nullable, device [S][max_iter]) per
 * iteration the index m of the accepted damping value or -1 (rejected);
 * entries past the last iteration are left untouched.  Saccades whose trace
 * holds NaN/Inf get NaN outputs.  Queued on `stream`; OPMM_EINVAL on bad
 * parameters or model not 9/18, before anything is queued. */
int opmm_polish(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                const opmm_polish_params* prm, int32_t model, float* opc_inout, float* rmse_out, float* mae_out,
                int32_t* iters_out, int8_t* decisions_out, void* stream);

/* ------------------------------------------------------------------------
 * Saccade extraction by velocity threshold (I-VT), the identification step
 * before estimation (Section 3.1; Section 4 uses I-VT and drops saccades
 * shorter than 6 ms).  gaze: device [N][2] FP32 positions (deg), sample
 * period dt_ms.  A sample k >= 1 is fast when |g_k - g_{k-1}| / dt exceeds
 * vel_thresh_deg_s; a saccade is a maximal run of fast samples, its trace
 * the run with the preceding (fixation) sample prepended, re-based to that
 * sample (T = run length + 1, duration (T-1) dt, amplitude and direction of
 * the last sample).  Runs with duration < min_dur_ms, amplitude <
 * min_amp_deg or T > max_T are dropped.  The output is the stream's first
 * saccades, in order, up to max_out records and pos_cap floats of trace (it
 * stops at the first saccade that does not fit): records to sacs_out
 * (HOST [max_out], pos_offset into pos_out,
 * seed = seed_base + first sample), traces to pos_out (device, pos_cap
 * floats, [T][2] back to back), src_start_out (HOST, nullable) = index of
 * each trace's first sample in the stream.  Ready for opmm_fit.  *n_out
 * (host) = saccades written.  Synchronises the stream.
 * ------------------------------------------------------------------------ */
int opmm_ivt_extract(opmm_ctx* ctx, const float* gaze, int64_t N, float dt_ms, float vel_thresh_deg_s,
                     float min_dur_ms, float min_amp_deg, int32_t max_T, uint64_t seed_base, int32_t max_out,
                     opmm_saccade* sacs_out, float* pos_out, int64_t pos_cap, int64_t* src_start_out,
                     int32_t* n_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* OPMM_H */
