// libopmm: OPMM estimation on MI355X (gfx950) -- kernels and the C ABI of
// include/opmm.h.
//
// Hot path (one fused kernel per candidate tile):
//   candidate draw (SplitMix64 stream, in registers)
//   -> per-candidate plant setup (D-form one-sample transition, equilibria)
//   -> T-sample recurrence with the projected target trace in LDS and the
//      squared residual accumulated on the fly
//   -> wave/block argmin of a packed (SSE bits, index) key -> one 64-bit
//      atomicMin per tile on the saccade's round slot.
// Candidates of a tile are ordered by the sample that holds their pulse end
// (a counting sort in LDS) before they are assigned to lanes, so the lanes of
// a wave switch from the pulse to the step within one or two samples of each
// other and the recurrence stays branch-free elsewhere.  The ordering changes
// nothing in any lane's arithmetic, and the argmin key is order-independent,
// so results are bit-identical for every tile shape and batch layout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/opmm.h"
#include "plant.hpp"
#include "runtime.hpp"

using namespace opmm;
using opmm_rt::KernelTimer;
using opmm_rt::SacDev;

namespace {

constexpr int NBIN = 256;  // pulse-end sample bins of the in-tile sort

#ifndef OPMM_MIN_WAVES
#define OPMM_MIN_WAVES 2  // waves per SIMD the register allocation must leave room for
#endif

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------

__global__ void fill_u64_kernel(uint64_t* p, int64_t n, uint64_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Project each trace on the movement direction: r_k = h cos + v sin, and the
// energy orthogonal to it, Q = sum (v cos - h sin)^2.  Then
// sum_k sum_c (pos - theta u)^2 = sum_k (r_k - theta_k)^2 + Q for every theta.
// One wave per saccade (block s): lanes take every 64th sample, then the
// wave combines Q and the finiteness flag.
__global__ __launch_bounds__(64) void prep_kernel(int S, const SacDev* __restrict__ sacs, const float* __restrict__ pos,
                                                  float* __restrict__ proj, double* __restrict__ qorth,
                                                  int32_t* __restrict__ status)
{
    const int s = blockIdx.x;
    if (s >= S) return;
    const SacDev sd = sacs[s];
    bool ok = true;
    double q = 0.0;
    for (int k = threadIdx.x; k < sd.T; k += 64) {
        double h = pos[sd.pos_off + (int64_t)k * sd.C];
        double v = sd.C == 2 ? (double)pos[sd.pos_off + (int64_t)k * sd.C + 1] : 0.0;
        ok = ok && isfinite(h) && isfinite(v);
        double r = h * sd.cphi + v * sd.sphi;
        if (sd.C == 2) {
            double o = v * sd.cphi - h * sd.sphi;
            q += o * o;
        }
        proj[sd.proj_off + k] = (float)r;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) q += __shfl_xor(q, o);
    ok = __all(ok);
    if (threadIdx.x == 0) {
        qorth[sd.slot] = q;
        status[sd.slot] = ok ? OPMM_ST_OK : OPMM_ST_NONFINITE_INPUT;
    }
}

// Round-0 box: centre = nominal (PW = D - 6), w = box_frac * centre, bounds
// centre -/+ w; optional seed centre (clamped) and narrower round-0 width.
__global__ void init_kernel(int S, const SacDev* __restrict__ sacs, float box_frac, float w_init_frac,
                            const float* __restrict__ seed_opc, float* __restrict__ centre,
                            float* __restrict__ hw, float* __restrict__ lo, float* __restrict__ hi,
                            int32_t* __restrict__ status)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S * P) return;
    int s = i / P, j = i % P;
    const int slot = sacs[s].slot;
    float c0 = nominal_param(j, sacs[s].dur);
    float w0 = (sacs[s].model == 9 && fixed_in_model9(j)) ? 0.0f : box_frac * c0;
    float l = c0 - w0, h = c0 + w0;
    float c = c0;
    if (seed_opc) {
        // 9-parameter model: tied components take the agonist's seed
        const int js = (sacs[s].model == 9 && (j == 1 || j == 3)) ? j - 1 : j;
        float v = seed_opc[(int64_t)s * P + js];
        c = (v == v) ? fminf(fmaxf(v, l), h) : c0;
        if (j == 0) status[slot] |= OPMM_ST_SEEDED;
    }
    const int64_t o = (int64_t)slot * P + j;
    centre[o] = c;
    hw[o] = w0 * w_init_frac;
    lo[o] = l;
    hi[o] = h;
}

__global__ void reset_keys_kernel(int n, const SacDev* __restrict__ sacs, uint64_t* keys)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keys[sacs[i].slot] = ~0ull;
}

__device__ __forceinline__ void load_box(Box& b, int s, const float* centre, const float* hw,
                                         const float* lo, const float* hi)
{
    for (int i = threadIdx.x; i < 4 * P; i += blockDim.x) {
        int a = i / P, j = i % P;
        const float* src = a == 0 ? centre : a == 1 ? hw : a == 2 ? lo : hi;
        float v = src[s * P + j];
        if (a == 0) b.c[j] = v;
        else if (a == 1) b.w[j] = v;
        else if (a == 2) b.lo[j] = v;
        else b.hi[j] = v;
    }
}

// next centre = winner of round r, half-width *= shrink (one thread / saccade)
__device__ __forceinline__ void refine_one(const SacDev& sd, int s, int r, uint64_t key, float shrink,
                                           float* centre, float* hw, const float* lo, const float* hi,
                                           int32_t* status)
{
    Box b;
    for (int j = 0; j < P; ++j) {
        b.c[j] = centre[s * P + j];
        b.w[j] = hw[s * P + j];
        b.lo[j] = lo[s * P + j];
        b.hi[j] = hi[s * P + j];
    }
    uint32_t idx = (uint32_t)(key & 0xFFFFFFFFull);
    if ((key >> 32) >= 0x7F800000ull) {
        atomicOr(&status[s], (int32_t)OPMM_ST_NO_FINITE_CANDIDATE);
        idx = 0;
    }
    float p[P];
    draw_candidate(sd.seed, (uint32_t)r, idx, b, p, sd.model);
    for (int j = 0; j < P; ++j) {
        centre[s * P + j] = p[j];
        hw[s * P + j] = b.w[j] * shrink;
    }
}

// round >= 0: every saccade is at that round and keys are [round][key_stride];
// round < 0: each saccade is at its own sd.round and keys are [slot].
__global__ void refine_kernel(int S, const SacDev* __restrict__ sacs, int round, int key_stride,
                              const uint64_t* __restrict__ keys, float shrink, float* centre, float* hw,
                              const float* lo, const float* hi, int32_t* status)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const SacDev sd = sacs[s];
    if (status[sd.slot] & OPMM_ST_NONFINITE_INPUT) return;
    const int r = round >= 0 ? round : sd.round;
    refine_one(sd, sd.slot, r, keys[(int64_t)(round >= 0 ? r : 0) * key_stride + sd.slot], shrink, centre, hw, lo,
               hi, status);
}

// ---------------------------------------------------------------------------
// Sinks for run_trajectory
// ---------------------------------------------------------------------------

template <class RT>
struct SseSinkT {  // squared residual against the projected trace in LDS, summed in Prec<RT>::acc
    using A = typename Prec<RT>::acc;
    const RT* r;
    A sse;
    __device__ __forceinline__ void operator()(int k, RT dth, RT theq)
    {
        RT e = (r[k] - theq) - dth;
        sse = fmr((A)e, (A)e, sse);
    }
};
using SseSink = SseSinkT<R>;

struct TrajSink {  // theta_k to global memory
    float* out;
    __device__ __forceinline__ void operator()(int k, R dth, R theq) { out[k] = (float)(dth + theq); }
};

struct Cost2dSink {  // both channels, FP64 accumulation (reporting only)
    const float* pos;
    int C;
    double cphi, sphi, sq, ab;
    __device__ __forceinline__ void operator()(int k, R dth, R theq)
    {
        double th = (double)(dth + theq);
        double e0 = (double)pos[(int64_t)k * C] - th * cphi;
        sq += e0 * e0;
        ab += fabs(e0);
        if (C == 2) {
            double e1 = (double)pos[(int64_t)k * C + 1] - th * sphi;
            sq += e1 * e1;
            ab += fabs(e1);
        }
    }
};

__device__ __forceinline__ uint64_t cost_key(double sse64, uint32_t idx)
{
    float sse = (float)sse64;
    float c = (sse >= 0.0f && sse <= 3.402823466e38f) ? sse : __int_as_float(0x7F800000);
    return ((uint64_t)__float_as_uint(c) << 32) | idx;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        uint64_t w = (uint64_t)__shfl_xor((unsigned long long)v, o);
        v = w < v ? w : v;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Fused tile: draw, sort by pulse-end sample, simulate + score, argmin
// ---------------------------------------------------------------------------

template <int TPB, int PASSES, class RT = R>
struct TileSmem {
    RT r[OPMM_MAX_T];
    Box box;
    int hist[NBIN];
    uint16_t perm[TPB * PASSES];
    uint64_t red[TPB / 64];
    int redv[TPB / 64];
};

// Returns the block's best key (valid in thread 0).  RT: the recurrence's precision (the screening
// pass runs it in FP32).  costs (nullable): for every slot q of the tile in pulse-end order, at
// [(tile_base + t) * TILE + q], the candidate's squared-residual sum rounded to FP32 (high word) and
// its index in the tile (low word), or all ones for a slot past the saccade's candidates.  tmin
// (with costs): at [tile_base + t], the bits of the tile's least FP32 sum, 0 if one is NaN, +inf
// if the tile holds no candidate.
template <int TPB, int PASSES, int UNROLL, class RT = R>
__device__ __forceinline__ uint64_t process_tile(TileSmem<TPB, PASSES, RT>& sm, const SacDev& sd, int s, int t,
                                                 int round, float dt, const float* __restrict__ proj,
                                                 const float* centre, const float* hw, const float* lo,
                                                 const float* hi, uint64_t* __restrict__ costs = nullptr,
                                                 uint32_t* __restrict__ tmin = nullptr)
{
    constexpr int TILE = TPB * PASSES;
    const int tid = threadIdx.x;
    const int T = sd.T;
    for (int k = tid; k < T; k += TPB) sm.r[k] = (RT)proj[sd.proj_off + k];
    load_box(sm.box, sd.slot, centre, hw, lo, hi);
    for (int i = tid; i < NBIN; i += TPB) sm.hist[i] = 0;
    __syncthreads();

    // Phase A: bin every candidate of the tile by its pulse-end sample.
    const uint32_t base = (uint32_t)t * TILE;
    const float rdt = rcp(dt);
    const float kbase = floorf(sm.box.lo[17] * rdt);
    int mybin[PASSES];
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
        uint32_t idx = base + ps * TPB + tid;
        int bin = NBIN - 1;
        if ((int64_t)idx < sd.n_cand) {
            float pw = draw_pw(sd.seed, (uint32_t)round, idx, sm.box) * rdt;
            float rel = fminf(fmaxf(floorf(pw) - kbase, 0.0f), (float)(NBIN - 2));
            bin = (int)rel;
        }
        mybin[ps] = bin;
        atomicAdd(&sm.hist[bin], 1);
    }
    __syncthreads();
    if (tid < 64) {  // exclusive scan of the histogram by wave 0
        int v[NBIN / 64];
        int run = 0;
#pragma unroll
        for (int i = 0; i < NBIN / 64; ++i) { v[i] = sm.hist[tid * (NBIN / 64) + i]; run += v[i]; }
        int incl = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int u = __shfl_up(incl, o);
            if (tid >= o) incl += u;
        }
        int acc = incl - run;
#pragma unroll
        for (int i = 0; i < NBIN / 64; ++i) { sm.hist[tid * (NBIN / 64) + i] = acc; acc += v[i]; }
    }
    __syncthreads();
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
        int slot = atomicAdd(&sm.hist[mybin[ps]], 1);
        sm.perm[slot] = (uint16_t)(ps * TPB + tid);
    }
    __syncthreads();

    // Phase B: simulate and score in sorted order.
    uint64_t best = ~0ull;
    int vmin = 0x7F800000;  // bits of the lane's least FP32 sum (non-negative floats order as integers)
#pragma unroll 1
    for (int ps = 0; ps < PASSES; ++ps) {
        // keep the box in LDS: re-read it per candidate instead of pinning 72 registers
        asm volatile("" ::: "memory");
        const uint32_t j = sm.perm[ps * TPB + tid];
        const uint32_t idx = base + j;
        const bool valid = (int64_t)idx < sd.n_cand;
        uint64_t* cslot = costs ? costs + (int64_t)(sd.tile_base + t) * TILE + ps * TPB + tid : nullptr;
        if (!__any(valid)) {
            if (cslot) *cslot = ~0ull;
            continue;
        }
        float p[P];
        draw_candidate(sd.seed, (uint32_t)round, idx, sm.box, p, sd.model);
        PlantT<RT> pl;
        plant_setup(p, sd.amp, dt, pl);
        RT frac;
        int k0 = pulse_end_sample(pl.pwd, T, frac);
        int kmin = wave_min(valid ? k0 : 0x7FFFFFFF);
        int kmax = wave_max(valid ? k0 : -0x7FFFFFFF);
        kmin = __builtin_amdgcn_readfirstlane(kmin);
        kmax = __builtin_amdgcn_readfirstlane(kmax);
        SseSinkT<RT> sink{sm.r, 0.0};
        if (valid) {
            run_trajectory<UNROLL>(pl, T, (RT)dt, k0, frac, kmin, kmax, sink);
            uint64_t key = cost_key(sink.sse, idx);
            best = key < best ? key : best;
        }
        if (cslot) {
            const float c = (float)sink.sse;
            *cslot = valid ? ((uint64_t)__float_as_uint(c) << 32) | j : ~0ull;
            if (valid) vmin = min(vmin, c != c ? 0 : (int)__float_as_uint(c));
        }
    }
    best = wave_min_u64(best);
    if (tmin) vmin = wave_min(vmin);
    if ((tid & 63) == 0) {
        sm.red[tid >> 6] = best;
        if (tmin) sm.redv[tid >> 6] = vmin;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < TPB / 64; ++w) best = sm.red[w] < best ? sm.red[w] : best;
        if (tmin) {
            for (int w = 1; w < TPB / 64; ++w) vmin = min(vmin, sm.redv[w]);
            tmin[sd.tile_base + t] = (uint32_t)vmin;
        }
    }
    return best;
}

// Last s with sacs[s].tile_base <= b (tile bases increase from 0), by one
// whole wave: each level probes 64 evenly spaced records at once and keeps the
// segment after the last probe that is <= b, so S = 4096 takes 2 dependent
// loads instead of 12.  Every lane of the wave must call it.
__device__ __forceinline__ int find_saccade_wave(const SacDev* __restrict__ sacs, int S, int b)
{
    const int lane = threadIdx.x & 63;
    int lo = 0, n = S;
    while (n > 1) {
        const int step = (n + 63) / 64;
        const bool le = lane * step < n && sacs[lo + lane * step].tile_base <= b;
        const uint64_t m = __ballot(le);  // lane 0 always set: sacs[lo].tile_base <= b
        const int last = 63 - __clzll((long long)m);
        lo += last * step;
        n = min(step, n - last * step);
    }
    return lo;
}

// Last k with base[k] <= b over a non-decreasing int array (base[0] = 0), by one
// whole wave, as find_saccade_wave.
__device__ __forceinline__ int find_index_wave(const int* __restrict__ base, int S, int b)
{
    const int lane = threadIdx.x & 63;
    int lo = 0, n = S;
    while (n > 1) {
        const int step = (n + 63) / 64;
        const bool le = lane * step < n && base[lo + lane * step] <= b;
        const uint64_t m = __ballot(le);
        const int last = 63 - __clzll((long long)m);
        lo += last * step;
        n = min(step, n - last * step);
    }
    return lo;
}

// Saccade of tile b.  ord (nullable): saccades in dispatch order (longest trace
// first, so the last blocks of a launch are short ones), obase their tile bases;
// without it, tiles follow the record order.  Every lane of the wave calls it.
__device__ __forceinline__ int saccade_of_tile(const SacDev* __restrict__ sacs, const int* __restrict__ ord,
                                               const int* __restrict__ obase, int S, int b)
{
    if (ord) return ord[find_index_wave(obase, S, b)];
    return find_saccade_wave(sacs, S, b);
}

// One round over a batch: round >= 0 puts every saccade at that round with keys
// [round][key_stride]; round < 0 takes each saccade's own round (sd.round) and
// keys [slot] (saccades admitted at different times, see the server).
template <int TPB, int PASSES, int UNROLL>
__global__ __launch_bounds__(TPB, OPMM_MIN_WAVES) void fit_round_kernel(const SacDev* __restrict__ sacs, int S, int round,
                                                        int key_stride, float dt, const float* __restrict__ proj,
                                                        const float* centre, const float* hw,
                                                        const float* lo, const float* hi,
                                                        const int32_t* __restrict__ status,
                                                        uint64_t* keys, const int* __restrict__ ord,
                                                        const int* __restrict__ obase)
{
    __shared__ TileSmem<TPB, PASSES> sm;
    __shared__ int s_s;
    if (threadIdx.x < 64) {
        const int sw = saccade_of_tile(sacs, ord, obase, S, blockIdx.x);
        if (threadIdx.x == 0) s_s = sw;
    }
    __syncthreads();
    const int s = s_s;
    const SacDev sd = sacs[s];
    if (status[sd.slot] & OPMM_ST_NONFINITE_INPUT) return;
    const int t = blockIdx.x - sd.tile_base;
    const int r = round >= 0 ? round : sd.round;
    uint64_t best = process_tile<TPB, PASSES, UNROLL>(sm, sd, s, t, r, dt, proj, centre, hw, lo, hi);
    if (threadIdx.x == 0 && best != ~0ull)
        atomicMin((unsigned long long*)&keys[(int64_t)(round >= 0 ? r : 0) * key_stride + sd.slot],
                  (unsigned long long)best);
}

// Screened round, first pass: the round's tiles with the recurrence in FP32.  Every candidate's
// squared-residual sum goes to costs; each saccade's FP32 best key to smin[slot].
// With its FP32 setup and the scaled Horner transition the FP32 pass needs 125 registers, so 4
// waves fit per SIMD; the bound only caps it at 168 (3 waves).  A 5-wave bound spills 23 registers.
#ifndef OPMM_SCREEN_MIN_WAVES
#define OPMM_SCREEN_MIN_WAVES 3
#endif
template <int TPB, int PASSES, int UNROLL>
__global__ __launch_bounds__(TPB, OPMM_SCREEN_MIN_WAVES) void fit_screen_kernel(const SacDev* __restrict__ sacs, int S,
                                                         int round, float dt, const float* __restrict__ proj,
                                                         const float* centre, const float* hw, const float* lo,
                                                         const float* hi, const int32_t* __restrict__ status,
                                                         const int* __restrict__ ord, const int* __restrict__ obase,
                                                         uint64_t* __restrict__ costs, uint32_t* __restrict__ tmin,
                                                         uint64_t* smin)
{
    __shared__ TileSmem<TPB, PASSES, float> sm;
    __shared__ int s_s;
    if (threadIdx.x < 64) {
        const int sw = saccade_of_tile(sacs, ord, obase, S, blockIdx.x);
        if (threadIdx.x == 0) s_s = sw;
    }
    __syncthreads();
    const SacDev sd = sacs[s_s];
    if (status[sd.slot] & OPMM_ST_NONFINITE_INPUT) return;
    const int t = blockIdx.x - sd.tile_base;
    const uint64_t best =
        process_tile<TPB, PASSES, UNROLL, float>(sm, sd, s_s, t, round, dt, proj, centre, hw, lo, hi, costs, tmin);
    if (threadIdx.x == 0 && best != ~0ull) atomicMin((unsigned long long*)&smin[sd.slot], (unsigned long long)best);
}

// Screened round, between the passes: one wave per saccade stages the trace in LDS, and its first
// lane re-simulates the FP32 pass's best candidate b in FP64, exactly as the round kernel would, and
// sets the verify threshold in SSE terms: FP32 RMSE <= RMSE64(b) + tau / 2.  The FP64 argmin x*
// passes it whenever the FP32 error eps stays below tau / 2: RMSE32(x*) <= RMSE64(x*) + eps <=
// RMSE64(b) + eps.  (With the FP32 best itself as the anchor the bound would need RMSE32(b) +
// 2 eps, a threshold about tau / 2 wider.)  The trace sits in dynamic LDS of max_T doubles.
extern __shared__ R anchor_trace[];

__global__ __launch_bounds__(64) void screen_anchor_kernel(const SacDev* __restrict__ sacs, int round, float dt,
                                                           const float* __restrict__ proj, const float* centre,
                                                           const float* hw, const float* lo, const float* hi,
                                                           const int32_t* __restrict__ status,
                                                           const double* __restrict__ qorth,
                                                           const uint64_t* __restrict__ smin, float tau, int max_T,
                                                           double* __restrict__ thr)
{
    __shared__ Box box;
    const SacDev sd = sacs[blockIdx.x];
    const int slot = sd.slot;
    const uint64_t key = smin[slot];
    const float fbest = __uint_as_float((uint32_t)(key >> 32));
    if ((status[slot] & OPMM_ST_NONFINITE_INPUT) || !(fbest <= 3.402823466e38f) || sd.T > max_T) {
        if (threadIdx.x == 0) thr[slot] = __builtin_inf();  // every candidate is verified
        return;
    }
    R* const r = anchor_trace;
    for (int k = threadIdx.x; k < sd.T; k += 64) r[k] = (R)proj[sd.proj_off + k];
    load_box(box, slot, centre, hw, lo, hi);
    __syncthreads();
    if (threadIdx.x != 0) return;
    float p[P];
    draw_candidate(sd.seed, (uint32_t)round, (uint32_t)key, box, p, sd.model);
    Plant pl;
    plant_setup(p, sd.amp, dt, pl);
    R frac;
    const int k0 = pulse_end_sample(pl.pwd, sd.T, frac);
    SseSink sink{r, 0.0};
    run_trajectory<1>(pl, sd.T, (R)dt, k0, frac, k0, k0, sink);
    const double n = (double)sd.T * sd.C, q = qorth[slot];
    const double rm = sqrt((sink.sse + q) / n) + 0.5 * (double)tau;
    thr[slot] = rm <= 1e300 ? rm * rm * n - q : __builtin_inf();  // a non-finite anchor verifies all
}

// Screened round, second pass, one wave per tile (a tile's survivors are often fewer than one
// block's lanes, and a one-wave block leaves no wave of it idle).  The tile's candidates whose FP32
// RMSE lies within tau of the saccade's FP32 best (or is NaN) are simulated again exactly as the FP64
// round kernel simulates them, in the first pass's pulse-end order, and their FP64 keys go to
// keys[round][slot].  The threshold comes from screen_anchor_kernel: with n = T C samples and Q the
// orthogonal energy, RMSE = sqrt((SSE + Q) / n), so a candidate passes when its FP32 SSE <=
// (RMSE64(b) + tau / 2)^2 n - Q.  A tile whose least FP32 SSE (tmin, 0 when one is NaN) misses that
// is left without reading its costs.
template <int TILE>
struct VerifySmem {
    Box box;
    uint16_t list[TILE];  // survivors' indices in the tile, in slot order
};
// The projected trace of the verifying wave's saccade, [max_T] of dynamic LDS (max_T: the batch's
// longest trace), so that short traces leave room for more waves per CU.
extern __shared__ R verify_trace[];

template <int TILE, int UNROLL>
__global__ __launch_bounds__(64, OPMM_MIN_WAVES) void fit_verify_kernel(
    const SacDev* __restrict__ sacs, int S, int round, int key_stride, float dt, const float* __restrict__ proj,
    const float* centre, const float* hw, const float* lo, const float* hi, const int32_t* __restrict__ status,
    uint64_t* keys, const int* __restrict__ ord, const int* __restrict__ obase, const uint64_t* __restrict__ costs,
    const uint32_t* __restrict__ tmin, const double* __restrict__ vthr, int max_T)
{
    static_assert(TILE % 64 == 0 && TILE <= 65536, "tile");
    constexpr int CH = TILE / 64;  // 64-slot chunks of the tile
    constexpr int PFV = CH < 8 ? CH : 8;  // chunks loaded ahead
    __shared__ VerifySmem<TILE> sm;
    const int lane = threadIdx.x;
    const int s = __builtin_amdgcn_readfirstlane(saccade_of_tile(sacs, ord, obase, S, blockIdx.x));
    const SacDev sd = sacs[s];
    if ((status[sd.slot] & OPMM_ST_NONFINITE_INPUT) || sd.T > max_T) return;  // max_T bounds the trace's LDS
    const int t = blockIdx.x - sd.tile_base;
    const int T = sd.T;
    const double thr = vthr[sd.slot];
    if (!((double)__uint_as_float(tmin[sd.tile_base + t]) <= thr)) return;
    // compaction in slot order, 64 slots at a time, PFV chunks of loads in flight
    const uint64_t* tc = costs + (int64_t)(sd.tile_base + t) * TILE + lane;
    uint64_t vals[PFV];
#pragma unroll
    for (int c = 0; c < PFV; ++c) vals[c] = tc[64 * c];
    int nv = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const uint64_t v = vals[c % PFV];
        if (c + PFV < CH) vals[c % PFV] = tc[64 * (c + PFV)];
        const uint32_t j = (uint32_t)v;
        const float f = __uint_as_float((uint32_t)(v >> 32));
        const bool pass = j != 0xFFFFFFFFu && ((double)f <= thr || f != f);
        const uint64_t m = __ballot(pass);
        if (pass) sm.list[nv + __popcll(m & ((1ull << lane) - 1))] = (uint16_t)j;
        nv += __popcll(m);
    }
    if (nv == 0) return;
    R* const r = verify_trace;
    for (int k = lane; k < T; k += 64) r[k] = (R)proj[sd.proj_off + k];
    load_box(sm.box, sd.slot, centre, hw, lo, hi);
    __syncthreads();
    const uint32_t base = (uint32_t)t * TILE;
    uint64_t best = ~0ull;
#pragma unroll 1
    for (int i0 = 0; i0 < nv; i0 += 64) {
        asm volatile("" ::: "memory");
        const int i = i0 + lane;
        const bool valid = i < nv;
        const uint32_t idx = base + (valid ? (uint32_t)sm.list[i] : 0u);
        float p[P];
        draw_candidate(sd.seed, (uint32_t)round, idx, sm.box, p, sd.model);
        Plant pl;
        plant_setup(p, sd.amp, dt, pl);
        R frac;
        int k0 = pulse_end_sample(pl.pwd, T, frac);
        int kmin = wave_min(valid ? k0 : 0x7FFFFFFF);
        int kmax = wave_max(valid ? k0 : -0x7FFFFFFF);
        kmin = __builtin_amdgcn_readfirstlane(kmin);
        kmax = __builtin_amdgcn_readfirstlane(kmax);
        SseSink sink{r, 0.0};
        if (valid) {
            run_trajectory<UNROLL>(pl, T, (R)dt, k0, frac, kmin, kmax, sink);
            const uint64_t key = cost_key(sink.sse, idx);
            best = key < best ? key : best;
        }
    }
    best = wave_min_u64(best);
    if (lane == 0 && best != ~0ull)
        atomicMin((unsigned long long*)&keys[(int64_t)round * key_stride + sd.slot], (unsigned long long)best);
}

// Every round of every saccade in one launch: a work queue of (round, tile)
// items in round-major order.  The block that finishes the last tile of a
// saccade's round refines that saccade and publishes the next round; a block
// that takes a tile of a later round waits for that.  Every item it can wait
// on was handed out earlier to a running block, so the queue always drains.
// The wait is bounded (wait_limit polls): a block that gives up does not
// search its tile, marks the saccade OPMM_ST_WAIT_TIMEOUT and counts the
// give-up in *errflag, and still counts the tile as done, so the queue drains
// and every block exits.
template <int TPB, int PASSES, int UNROLL>
__global__ __launch_bounds__(TPB, OPMM_MIN_WAVES) void fit_persistent_kernel(
    const SacDev* __restrict__ sacs, int S, int R, int tiles_per_round, float dt, float shrink,
    const float* __restrict__ proj, float* centre, float* hw, const float* lo, const float* hi,
    int32_t* status, uint64_t* keys, uint32_t* head, uint32_t* done, uint32_t* ready, uint32_t* errflag,
    const int* __restrict__ ord, const int* __restrict__ obase, uint32_t wait_limit)
{
    __shared__ TileSmem<TPB, PASSES> sm;
    __shared__ int s_item, s_sac, s_gaveup;
    const int64_t total = (int64_t)R * tiles_per_round;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(head, 1u);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= total) break;
        const int r = (int)(item / tiles_per_round);
        const int b = (int)(item % tiles_per_round);
        if (threadIdx.x < 64) {
            const int sw = saccade_of_tile(sacs, ord, obase, S, b);
            if (threadIdx.x == 0) {
                s_sac = sw;
                s_gaveup = 0;
            }
        }
        __syncthreads();
        const int s = s_sac;
        const SacDev sd = sacs[s];
        const int t = b - sd.tile_base;
        const bool skip = (status[s] & OPMM_ST_NONFINITE_INPUT) != 0;
        if (!skip) {
            if (r > 0) {
                if (threadIdx.x == 0) {
                    bool ok = false;
                    for (uint32_t polls = 0; polls < wait_limit; ++polls) {
                        if (__hip_atomic_load(&ready[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= (uint32_t)r) {
                            ok = true;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                    if (!ok) {
                        s_gaveup = 1;
                        atomicAdd(errflag, 1u);
                        atomicOr(&status[s], (int32_t)OPMM_ST_WAIT_TIMEOUT);
                    }
                }
                __syncthreads();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            uint64_t best = ~0ull;
            if (!s_gaveup) best = process_tile<TPB, PASSES, UNROLL>(sm, sd, s, t, r, dt, proj, centre, hw, lo, hi);
            if (threadIdx.x == 0) {
                if (best != ~0ull)
                    atomicMin((unsigned long long*)&keys[(int64_t)r * S + s], (unsigned long long)best);
                __threadfence();
                uint32_t old = atomicAdd(&done[s], 1u);
                if (old + 1 == (uint32_t)((r + 1) * sd.tiles)) {
                    __threadfence();
                    uint64_t key = __hip_atomic_load(&keys[(int64_t)r * S + s], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                    refine_one(sd, s, r, key, shrink, centre, hw, lo, hi, status);
                    __threadfence();
                    __hip_atomic_store(&ready[s], (uint32_t)(r + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        __syncthreads();
    }
}

// After a persistent launch: add its give-up count to the context's report
// (read and cleared by opmm_sync).
__global__ void harvest_giveups_kernel(const uint32_t* __restrict__ errflag, uint32_t* report)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t n = *errflag;
        if (n) atomicAdd(report, n);
    }
}

// Final report: re-simulate each saccade's winner and score it on the full
// 2-channel trace (RMSE and mean absolute difference), FP64 accumulation.
// One wave per saccade (block s): the wave stages the trace in LDS, every
// lane runs the same simulation and lane 0 writes the results.
__global__ __launch_bounds__(64) void report_kernel(int S, const SacDev* __restrict__ sacs, const float* __restrict__ pos,
                                                    float dt, const float* __restrict__ centre, float* opc_out,
                                                    float* rmse_out, float* mae_out, const int32_t* __restrict__ status,
                                                    int32_t* status_out)
{
    __shared__ float tr[2 * OPMM_MAX_T];
    const int s = blockIdx.x;
    if (s >= S) return;
    const SacDev sd = sacs[s];
    for (int i = threadIdx.x; i < sd.T * sd.C; i += 64) tr[i] = pos[sd.pos_off + i];
    __syncthreads();
    float p[P];
    for (int j = 0; j < P; ++j) p[j] = centre[(int64_t)sd.slot * P + j];
    Plant pl;
    plant_setup(p, sd.amp, dt, pl);
    R frac;
    int k0 = pulse_end_sample(pl.pwd, sd.T, frac);
    Cost2dSink sink{tr, sd.C, sd.cphi, sd.sphi, 0.0, 0.0};
    run_trajectory<1>(pl, sd.T, (R)dt, k0, frac, k0, k0, sink);
    if (threadIdx.x != 0) return;
    const int32_t st = status[sd.slot];
    const bool bad = (st & OPMM_ST_NONFINITE_INPUT) != 0;
    const double n = (double)sd.T * sd.C;
    for (int j = 0; j < P; ++j) opc_out[s * P + j] = bad ? __int_as_float(0x7FC00000) : p[j];
    double rm = sqrt(sink.sq / n);
    rmse_out[s] = bad ? __int_as_float(0x7FC00000) : (float)rm;
    if (mae_out) mae_out[s] = bad ? __int_as_float(0x7FC00000) : (float)(sink.ab / n);
    if (status_out) status_out[s] = st;
}

// ---------------------------------------------------------------------------
// Standalone simulate / score / candidates
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256, OPMM_MIN_WAVES) void simulate_kernel(int64_t n, const float* __restrict__ opc,
                                                       const float* __restrict__ amp, int T, float dt,
                                                       float* __restrict__ traj)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = i < n;
    int64_t ii = valid ? i : 0;
    float p[P];
    for (int j = 0; j < P; ++j) p[j] = opc[ii * P + j];
    Plant pl;
    plant_setup(p, amp[ii], dt, pl);
    R frac;
    int k0 = pulse_end_sample(pl.pwd, T, frac);
    int kmin = wave_min(valid ? k0 : 0x7FFFFFFF), kmax = wave_max(valid ? k0 : -0x7FFFFFFF);
    if (!valid) return;
    TrajSink sink{traj + ii * T};
    run_trajectory<2>(pl, T, (R)dt, k0, frac, kmin, kmax, sink);
}

// RMSE of n candidates against one saccade, with the recurrence of precision RT (FP64: the search's
// decisions; FP32: the screening pass's arithmetic, sample by sample the same operations).
template <class RT>
__global__ __launch_bounds__(256, OPMM_MIN_WAVES) void score_kernel(int64_t n, const float* __restrict__ opc,
                                                    const float* __restrict__ proj, int T, int C,
                                                    const double* __restrict__ qorth, float amp, float dt,
                                                    float* __restrict__ rmse)
{
    __shared__ RT r[OPMM_MAX_T];
    for (int k = threadIdx.x; k < T; k += blockDim.x) r[k] = (RT)proj[k];
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = i < n;
    int64_t ii = valid ? i : 0;
    float p[P];
    for (int j = 0; j < P; ++j) p[j] = opc[ii * P + j];
    PlantT<RT> pl;
    plant_setup(p, amp, dt, pl);
    RT frac;
    int k0 = pulse_end_sample(pl.pwd, T, frac);
    int kmin = wave_min(valid ? k0 : 0x7FFFFFFF), kmax = wave_max(valid ? k0 : -0x7FFFFFFF);
    if (!valid) return;
    SseSinkT<RT> sink{r, 0.0};
    run_trajectory<2>(pl, T, (RT)dt, k0, frac, kmin, kmax, sink);
    double tot = ((double)sink.sse + qorth[0]) / ((double)T * C);
    float v = (float)sqrt(tot);
    rmse[i] = (v >= 0.0f && v <= 3.402823466e38f) ? v : __int_as_float(0x7F800000);
}

struct BoxArg {
    float v[4][P];
};

__global__ void candidates_kernel(uint64_t seed, uint32_t round, uint32_t idx0, int64_t n, BoxArg ba,
                                  float* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Box b;
    for (int j = 0; j < P; ++j) {
        b.c[j] = ba.v[0][j]; b.w[j] = ba.v[1][j]; b.lo[j] = ba.v[2][j]; b.hi[j] = ba.v[3][j];
    }
    float p[P];
    draw_candidate(seed, round, idx0 + (uint32_t)i, b, p);
    for (int j = 0; j < P; ++j) out[i * P + j] = p[j];
}

// ---------------------------------------------------------------------------
// Kernel shapes
// ---------------------------------------------------------------------------

struct Shape {
    int tpb, passes, unroll;
    const char* name;
};
const Shape kShapes[] = {
    {256, 4, 1, "tpb256_pass4_unroll1"},
    {256, 2, 1, "tpb256_pass2_unroll1"},
    {256, 8, 1, "tpb256_pass8_unroll1"},
    {128, 8, 1, "tpb128_pass8_unroll1"},
    {256, 4, 2, "tpb256_pass4_unroll2"},
    {256, 4, 4, "tpb256_pass4_unroll4"},
    {64, 16, 1, "tpb64_pass16_unroll1"},
    {256, 16, 1, "tpb256_pass16_unroll1"},
    {128, 32, 1, "tpb128_pass32_unroll1"},
    {256, 8, 4, "tpb256_pass8_unroll4"},
    {256, 4, 8, "tpb256_pass4_unroll8"},
    {64, 16, 4, "tpb64_pass16_unroll4"},
    {128, 8, 4, "tpb128_pass8_unroll4"},
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
constexpr int kDefaultShape = 9;  // fastest per-round shape on the full-estimation workload (sweep)

struct FitLaunch {
    const SacDev* sacs;
    int S, R, tiles_per_round;
    int key_stride;
    float dt, shrink;
    const float* proj;
    float *centre, *hw, *lo, *hi;
    int32_t* status;
    uint64_t* keys;
    uint32_t *head, *done, *ready, *errflag;
    int grid_persistent;
    const int *ord, *obase;  // dispatch order (nullable: record order)
    uint32_t wait_limit;     // polls of a persistent block waiting for its round
    // screened rounds: FP32 costs of every candidate, FP32 best per saccade, orthogonal energies
    uint64_t* costs;  // [tiles_per_round * tile]: FP32 cost and index of every slot (process_tile)
    uint32_t* tmin;   // [tiles_per_round]: least FP32 cost of each tile (process_tile)
    int max_T;        // longest trace of the batch (0: unknown, OPMM_MAX_T assumed)
    uint64_t* smin;   // [S]: FP32 best key per saccade
    double* vthr;     // [S]: verify threshold per saccade (SSE units, screen_anchor_kernel)
    const double* qorth;
    float tau;
    KernelTimer* timer;  // non-null: record an event pair around each search-kernel launch
};

// Event pair around one launch when the call is timed (see KernelTimer).
struct TimedLaunch {
    KernelTimer* t;
    int kernel, slot;
    hipStream_t st;
    TimedLaunch(KernelTimer* timer, int k, hipStream_t s) : t(timer), kernel(k), slot(-1), st(s)
    {
        if (t) slot = t->begin(st);
    }
    ~TimedLaunch()
    {
        if (t) t->end(kernel, slot, st);
    }
};

template <int TPB, int PASSES, int UNROLL>
hipError_t launch_shape(const FitLaunch& L, bool persistent, int round, hipStream_t st)
{
    TimedLaunch tl(L.timer, persistent ? OPMM_KERNEL_PERSISTENT : OPMM_KERNEL_ROUND, st);
    if (persistent) {
        hipLaunchKernelGGL((fit_persistent_kernel<TPB, PASSES, UNROLL>), dim3(L.grid_persistent), dim3(TPB), 0,
                           st, L.sacs, L.S, L.R, L.tiles_per_round, L.dt, L.shrink, L.proj, L.centre, L.hw,
                           L.lo, L.hi, L.status, L.keys, L.head, L.done, L.ready, L.errflag, L.ord, L.obase,
                           L.wait_limit);
    } else {
        hipLaunchKernelGGL((fit_round_kernel<TPB, PASSES, UNROLL>), dim3(L.tiles_per_round), dim3(TPB), 0, st,
                           L.sacs, L.S, round, L.key_stride, L.dt, L.proj, L.centre, L.hw, L.lo, L.hi, L.status,
                           L.keys, L.ord, L.obase);
    }
    return hipGetLastError();
}

template <int TPB, int PASSES, int UNROLL>
hipError_t launch_screened(const FitLaunch& L, int round, hipStream_t st)
{
    {
        TimedLaunch tl(L.timer, OPMM_KERNEL_SCREEN, st);
        hipLaunchKernelGGL((fit_screen_kernel<TPB, PASSES, UNROLL>), dim3(L.tiles_per_round), dim3(TPB), 0, st,
                           L.sacs, L.S, round, L.dt, L.proj, L.centre, L.hw, L.lo, L.hi, L.status, L.ord, L.obase,
                           L.costs, L.tmin, L.smin);
    }
    const int max_T = L.max_T > 0 && L.max_T <= OPMM_MAX_T ? L.max_T : OPMM_MAX_T;
    hipLaunchKernelGGL(screen_anchor_kernel, dim3(L.S), dim3(64), sizeof(R) * (size_t)max_T, st, L.sacs, round,
                       L.dt, L.proj, L.centre, L.hw, L.lo, L.hi, L.status, L.qorth, L.smin, L.tau, max_T, L.vthr);
    {
        TimedLaunch tl(L.timer, OPMM_KERNEL_VERIFY, st);
        hipLaunchKernelGGL((fit_verify_kernel<TPB * PASSES, UNROLL>), dim3(L.tiles_per_round), dim3(64),
                           sizeof(R) * (size_t)max_T, st, L.sacs, L.S, round, L.key_stride, L.dt, L.proj, L.centre,
                           L.hw, L.lo, L.hi, L.status, L.keys, L.ord, L.obase, L.costs, L.tmin, L.vthr, max_T);
    }
    return hipGetLastError();
}

// One screened round (FP32 pass + FP64 verification) of shape `shape`.
hipError_t launch_screened_round(int shape, const FitLaunch& L, int round, hipStream_t st)
{
    switch (shape) {
    case 0: return launch_screened<256, 4, 1>(L, round, st);
    case 1: return launch_screened<256, 2, 1>(L, round, st);
    case 2: return launch_screened<256, 8, 1>(L, round, st);
    case 3: return launch_screened<128, 8, 1>(L, round, st);
    case 4: return launch_screened<256, 4, 2>(L, round, st);
    case 5: return launch_screened<256, 4, 4>(L, round, st);
    case 6: return launch_screened<64, 16, 1>(L, round, st);
    case 7: return launch_screened<256, 16, 1>(L, round, st);
    case 8: return launch_screened<128, 32, 1>(L, round, st);
    case 9: return launch_screened<256, 8, 4>(L, round, st);
    case 10: return launch_screened<256, 4, 8>(L, round, st);
    case 11: return launch_screened<64, 16, 4>(L, round, st);
    default: return launch_screened<128, 8, 4>(L, round, st);
    }
}

hipError_t launch_fit_kernel(int shape, const FitLaunch& L, bool persistent, int round, hipStream_t st)
{
    switch (shape) {
    case 0: return launch_shape<256, 4, 1>(L, persistent, round, st);
    case 1: return launch_shape<256, 2, 1>(L, persistent, round, st);
    case 2: return launch_shape<256, 8, 1>(L, persistent, round, st);
    case 3: return launch_shape<128, 8, 1>(L, persistent, round, st);
    case 4: return launch_shape<256, 4, 2>(L, persistent, round, st);
    case 5: return launch_shape<256, 4, 4>(L, persistent, round, st);
    case 6: return launch_shape<64, 16, 1>(L, persistent, round, st);
    case 7: return launch_shape<256, 16, 1>(L, persistent, round, st);
    case 8: return launch_shape<128, 32, 1>(L, persistent, round, st);
    case 9: return launch_shape<256, 8, 4>(L, persistent, round, st);
    case 10: return launch_shape<256, 4, 8>(L, persistent, round, st);
    case 11: return launch_shape<64, 16, 4>(L, persistent, round, st);
    default: return launch_shape<128, 8, 4>(L, persistent, round, st);
    }
}

template <int TPB, int PASSES, int UNROLL>
int persistent_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit_persistent_kernel<TPB, PASSES, UNROLL>, TPB, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

int shape_blocks_per_cu(int shape)
{
    switch (shape) {
    case 0: return persistent_blocks_per_cu<256, 4, 1>();
    case 1: return persistent_blocks_per_cu<256, 2, 1>();
    case 2: return persistent_blocks_per_cu<256, 8, 1>();
    case 3: return persistent_blocks_per_cu<128, 8, 1>();
    case 4: return persistent_blocks_per_cu<256, 4, 2>();
    case 5: return persistent_blocks_per_cu<256, 4, 4>();
    case 6: return persistent_blocks_per_cu<64, 16, 1>();
    case 7: return persistent_blocks_per_cu<256, 16, 1>();
    case 8: return persistent_blocks_per_cu<128, 32, 1>();
    case 9: return persistent_blocks_per_cu<256, 8, 4>();
    case 10: return persistent_blocks_per_cu<256, 4, 8>();
    case 11: return persistent_blocks_per_cu<64, 16, 4>();
    default: return persistent_blocks_per_cu<128, 8, 4>();
    }
}

// ---------------------------------------------------------------------------
// Device scratch of one fit
// ---------------------------------------------------------------------------

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

struct FitScratch {
    DevBuf sacs, proj, qorth, box, keys, status, counters, order;
    DevBuf costs, tmin, smin, vthr;  // screened rounds (see FitBufs)
    int max_T = 0;             // longest trace of the last uploaded batch
    // Pinned host staging of the record upload (records, then dispatch order and tile bases), kept
    // between calls: the upload is a direct DMA and no batch pays for fresh pages.
    DevBuf stage;
    std::vector<int> h_count;
    ~FitScratch()
    {
        for (DevBuf* b : {&sacs, &proj, &qorth, &box, &keys, &status, &counters, &order, &costs, &tmin, &smin, &vthr})
            if (b->p) (void)hipFree(b->p);
        if (stage.p) (void)hipHostFree(stage.p);
    }
};

}  // namespace

// Device scratch of opmm_fit_noalloc: one array per device, held until the
// process ends.  Host code uses the address opmm_create looked up, never this name.
static __device__ __align__(256) unsigned char scratch[OPMM_NOALLOC_SCRATCH_BYTES];

// Autotuner cache key: what decides which kernel shape is fastest for a batch.
struct TuneKey {
    int mode, model;
    int t_bucket, s_bucket;  // longest trace and batch size, each rounded up to a power of two
    int64_t n_cand;          // largest candidate count in the batch
    bool operator==(const TuneKey& o) const
    {
        return mode == o.mode && model == o.model && t_bucket == o.t_bucket && s_bucket == o.s_bucket &&
               n_cand == o.n_cand;
    }
};
struct TuneEntry {
    TuneKey key;
    int shape;
    float ms;
};

struct opmm_ctx {
    int device = 0;
    std::string arch;                 // device architecture name (autotuner cache files are per architecture)
    std::vector<TuneEntry> tune;      // autotuner picks by batch key
    int cu_count = 0;
    uint32_t wait_limit = 1u << 26;        // polls before a persistent block gives up (several seconds)
    uint32_t* giveup_report = nullptr;     // device word: give-ups since the last opmm_sync
    std::string err;
    FitScratch scratch;
    FitScratch aux;  // projections for the learned seed, independent of the fit's scratch
    float* d_cand = nullptr;  // small per-call staging for opmm_score (projected trace)
    size_t d_cand_cap = 0;
    int tuned_shape = -1;
    hipStream_t cap_stream = nullptr;
    unsigned char* noalloc_scratch = nullptr;  // device address of `scratch` on this device (set at creation)
    opmm_rt::StreamOrder order;  // orders calls on different streams (scratch, aux, d_cand, give-up word)
    KernelTimer timer;           // per-kernel timing of uncaptured fits (off unless switched on)
};

struct opmm_plan {
    opmm_ctx* ctx = nullptr;
    FitScratch scratch;
    opmm_rt::StreamOrder order;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace opmm_rt {

int fail(opmm_ctx* ctx, int code, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(opmm_ctx* ctx, hipError_t e, const char* what)
{
    return fail(ctx, OPMM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

hipError_t order_init(StreamOrder& o) { return hipEventCreateWithFlags(&o.ev, hipEventDisableTiming); }

void order_release(StreamOrder& o)
{
    if (o.ev) (void)hipEventDestroy(o.ev);
    o.ev = nullptr;
    o.recorded = false;
}

hipError_t order_host_wait(const StreamOrder& o, hipStream_t st)
{
    if (o.ev && o.recorded) return hipEventSynchronize(o.ev);
    if (o.seen && o.last != st) return hipDeviceSynchronize();  // one stream so far, not this one
    return hipSuccess;
}

Ordered::Ordered(StreamOrder& o, hipStream_t st) : o_(o), st_(st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    err_ = hipStreamIsCapturing(st, &cs);
    skip_ = !o.ev || err_ != hipSuccess || cs != hipStreamCaptureStatusNone;
    if (skip_) return;
    if (o.seen && st != o.last) {
        if (!o.multi) {
            // no event marks the earlier calls: wait for all of them once, then record from now on
            err_ = hipDeviceSynchronize();
            o.multi = true;
        } else if (o.recorded) {
            err_ = hipStreamWaitEvent(st, o.ev, 0);
        }
    }
    o.seen = true;
    if (err_ != hipSuccess) skip_ = true;
}

Ordered::~Ordered()
{
    if (skip_) return;
    o_.last = st_;
    if (!o_.multi) return;
    if (hipEventRecord(o_.ev, st_) == hipSuccess)
        o_.recorded = true;
    else
        (void)hipGetLastError();
}

int ctx_device(const opmm_ctx* ctx) { return ctx ? ctx->device : 0; }
StreamOrder& ctx_order(opmm_ctx* ctx) { return ctx->order; }
int ctx_cu_count(const opmm_ctx* ctx) { return ctx && ctx->cu_count > 0 ? ctx->cu_count : 256; }

}  // namespace opmm_rt

namespace {

using opmm_rt::fail;
using opmm_rt::hip_fail;

#define OPMM_HIP(ctx, call)                                  \
    do {                                                     \
        hipError_t _e = (call);                              \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #call); \
    } while (0)

int ensure(opmm_ctx* ctx, DevBuf& b, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return OPMM_OK;
    if (b.p) {
        OPMM_HIP(ctx, hipDeviceSynchronize());
        OPMM_HIP(ctx, hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t cap = std::max(bytes, b.cap * 2);
    if (hipMalloc(&b.p, cap) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(ctx, OPMM_ENOMEM, "device allocation of " + std::to_string(cap) + " bytes failed");
    }
    b.cap = cap;
    return OPMM_OK;
}

// Grow a pinned host buffer.  Its previous contents are dead: every upload waits for its copies.
int ensure_host(opmm_ctx* ctx, DevBuf& b, size_t bytes)
{
    if (b.cap >= bytes) return OPMM_OK;
    if (b.p) {
        OPMM_HIP(ctx, hipHostFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t cap = std::max(bytes, b.cap * 2);
    if (hipHostMalloc(&b.p, cap, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(ctx, OPMM_ENOMEM, "pinned host allocation of " + std::to_string(cap) + " bytes failed");
    }
    b.cap = cap;
    return OPMM_OK;
}

int blocks_for(int64_t n, int tpb) { return (int)((n + tpb - 1) / tpb); }

// The reason a record is unusable, or nullptr (no string work on the accepted path: batches of
// thousands of records are checked on every call).
const char* saccade_defect(const opmm_saccade& s, int64_t pos_len)
{
    if (s.T < 1 || s.T > OPMM_MAX_T) return "T out of range";
    if (s.C != 1 && s.C != 2) return "C must be 1 or 2";
    if (s.C == 1 && !(s.dir_deg == 0.0f || s.dir_deg == 180.0f)) return "C = 1 needs dir_deg 0 or 180";
    if (!std::isfinite(s.amp_deg) || s.amp_deg < 0.0f) return "amp_deg must be finite and >= 0";
    if (!std::isfinite(s.dir_deg)) return "dir_deg must be finite";
    if (!std::isfinite(s.dur_ms) || !(s.dur_ms > 6.0f)) return "dur_ms must be > 6";
    if (s.pos_offset < 0 || s.pos_offset + (int64_t)s.T * s.C > pos_len) return "trace lies outside pos[0, pos_len)";
    if (s.n_cand < 0) return "n_cand must be >= 0";
    return nullptr;
}

int validate_saccade_impl(opmm_ctx* ctx, const opmm_saccade& s, int64_t pos_len, int i)
{
    const char* why = saccade_defect(s, pos_len);
    if (!why) return OPMM_OK;
    return fail(ctx, OPMM_EINVAL, std::string(why) + " (saccade " + std::to_string(i) + ")");
}

int validate_params(opmm_ctx* ctx, const opmm_fit_params* p)
{
    if (!p) return fail(ctx, OPMM_EINVAL, "params is NULL");
    if (p->n_cand < 1) return fail(ctx, OPMM_EINVAL, "n_cand must be >= 1");
    if (p->n_rounds < 1 || p->n_rounds > 4096) return fail(ctx, OPMM_EINVAL, "n_rounds must be in 1..4096");
    if (!(p->box_frac > 0.0f && p->box_frac < 1.0f)) return fail(ctx, OPMM_EINVAL, "box_frac must be in (0, 1)");
    if (!(p->w_init_frac >= 0.0f && p->w_init_frac <= 1.0f)) return fail(ctx, OPMM_EINVAL, "w_init_frac must be in [0, 1]");
    if (!(p->shrink > 0.0f && p->shrink <= 1.0f)) return fail(ctx, OPMM_EINVAL, "shrink must be in (0, 1]");
    if (!(p->dt_ms > 0.0f && p->dt_ms <= 1.0f)) return fail(ctx, OPMM_EINVAL, "dt_ms must be in (0, 1]");
    if (p->mode != OPMM_FIT_ROUNDS && p->mode != OPMM_FIT_PERSISTENT) return fail(ctx, OPMM_EINVAL, "bad mode");
    if (p->tile < -1 || p->tile >= kNumShapes) return fail(ctx, OPMM_EINVAL, "bad tile index");
    if (p->model != 18 && p->model != 9) return fail(ctx, OPMM_EINVAL, "model must be 18 or 9");
    if (p->screen_rounds < 0 || p->screen_rounds > p->n_rounds)
        return fail(ctx, OPMM_EINVAL, "screen_rounds must be in 0..n_rounds");
    if (p->screen_rounds > 0 && p->mode != OPMM_FIT_ROUNDS)
        return fail(ctx, OPMM_EINVAL, "screened rounds need the per-round mode");
    if (p->screen_rounds > 0 && !(p->screen_tol > 0.0f && p->screen_tol <= 3.402823466e38f))
        return fail(ctx, OPMM_EINVAL, "screen_tol must be positive and finite");
    return OPMM_OK;
}

// Host records of a batch (no allocation): h[S] device records, ob[2S] the
// dispatch order and each ordered saccade's first tile, cnt[OPMM_MAX_T + 1]
// counting scratch.  Returns the summed trace length and tile count.
void build_records(const opmm_saccade* sacs, int S, const opmm_fit_params* prm, int tile_size, SacDev* h, int* ob,
                   int* cnt, int64_t* total_T, int64_t* tiles_out)
{
    int64_t toff = 0;
    for (int i = 0; i < S; ++i) {
        SacDev& d = h[i];
        d = opmm_rt::make_record(sacs[i], prm ? prm->n_cand : 1);
        d.model = prm ? prm->model : 18;
        d.proj_off = toff;
        d.tiles = (int)((d.n_cand + tile_size - 1) / tile_size);
        d.slot = i;
        toff += sacs[i].T;
    }
    // Tiles are dispatched longest trace first (a tile's time grows with T), so a launch ends on
    // short blocks; ord[k] is the k-th saccade in that order and obase[k] its first tile.  The
    // order changes only which block takes a tile, never a result.  T is bounded, so a counting
    // sort on (OPMM_MAX_T - T) gives the order in O(S), ties in batch order.
    for (int k = 0; k <= OPMM_MAX_T; ++k) cnt[k] = 0;
    for (int i = 0; i < S; ++i) cnt[OPMM_MAX_T - sacs[i].T]++;  // T in 1..OPMM_MAX_T (validated)
    for (int k = 0, run = 0; k <= OPMM_MAX_T; ++k) {
        const int c = cnt[k];
        cnt[k] = run;
        run += c;
    }
    for (int i = 0; i < S; ++i) ob[cnt[OPMM_MAX_T - sacs[i].T]++] = i;
    int64_t tiles = 0;
    for (int k = 0; k < S; ++k) {
        SacDev& d = h[ob[k]];
        d.tile_base = (int)tiles;
        ob[S + k] = (int)tiles;
        tiles += d.tiles;
    }
    *total_T = toff;
    *tiles_out = tiles;
}

// Host records -> device records, prefix sums of tiles; uploads synchronously
// (the records are small) so the caller's host array can be reused at once.
int upload_saccades(opmm_ctx* ctx, FitScratch& sc, const opmm_saccade* sacs, int S,
                    const opmm_fit_params* prm, int tile_size, int64_t* total_T, int* tiles_per_round,
                    hipStream_t st)
{
    int rc;
    const size_t rec_bytes = sizeof(SacDev) * (size_t)S, ord_bytes = sizeof(int) * 2 * (size_t)S;
    if ((rc = ensure_host(ctx, sc.stage, rec_bytes + ord_bytes)) != OPMM_OK) return rc;
    static_assert(sizeof(SacDev) % alignof(int) == 0, "the order array follows the records");
    SacDev* h = (SacDev*)sc.stage.p;
    int* ob = (int*)((char*)sc.stage.p + rec_bytes);
    sc.h_count.resize(OPMM_MAX_T + 1);
    int64_t toff, tiles;
    build_records(sacs, S, prm, tile_size, h, ob, sc.h_count.data(), &toff, &tiles);
    if (tiles > 0x7FFFFFFF / 8) return fail(ctx, OPMM_EINVAL, "too many candidate tiles in one batch");
    sc.max_T = S > 0 ? sacs[ob[0]].T : 0;  // the dispatch order is longest trace first
    if ((rc = ensure(ctx, sc.sacs, rec_bytes)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.order, ord_bytes)) != OPMM_OK) return rc;
    OPMM_HIP(ctx, hipMemcpyAsync(sc.sacs.p, h, rec_bytes, hipMemcpyHostToDevice, st));
    OPMM_HIP(ctx, hipMemcpyAsync(sc.order.p, ob, ord_bytes, hipMemcpyHostToDevice, st));
    OPMM_HIP(ctx, hipStreamSynchronize(st));
    *total_T = toff;
    *tiles_per_round = (int)tiles;
    return OPMM_OK;
}

// Device buffers of one fit (sizes for S saccades, summed length total_T, R
// rounds): records [S], dispatch order [2S], projected traces [total_T], orthogonal
// energies [S], box [4][S][18], status [S], counters [2S + 2], round keys [R][S].
struct FitBufs {
    SacDev* sacs;
    int* order;
    float* proj;
    double* qorth;
    float* box;
    int32_t* status;
    uint32_t* counters;
    uint64_t* keys;
    // screened rounds only: FP32 cost and index of every candidate slot [tiles_per_round * tile],
    // least FP32 cost per tile [tiles_per_round], FP32 best key per saccade [S]
    uint64_t* costs = nullptr;
    uint32_t* tmin = nullptr;
    uint64_t* smin = nullptr;
    double* vthr = nullptr;  // verify threshold per saccade [S]
    int max_T = 0;  // longest trace (0: unknown)
};

int enqueue_fit_bufs(opmm_ctx* ctx, const FitBufs& B, const float* pos, int S, int tiles_per_round,
                     const opmm_fit_params* prm, int shape, const float* seed_opc, float* opc_out, float* rmse_out,
                     float* mae_out, int32_t* status_out, hipStream_t st, bool run_prep);

// Queue the whole fit on `st` (no host synchronisation inside: capturable).
// run_prep = false: the projection of this upload is already queued (fit_stage).
int enqueue_fit(opmm_ctx* ctx, FitScratch& sc, const float* pos, int S, int64_t total_T, int tiles_per_round,
                const opmm_fit_params* prm, int shape, const float* seed_opc, float* opc_out, float* rmse_out,
                float* mae_out, int32_t* status_out, uint64_t* round_keys, hipStream_t st, bool run_prep = true)
{
    const int R = prm->n_rounds;
    int rc;
    if ((rc = ensure(ctx, sc.proj, sizeof(float) * total_T)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.qorth, sizeof(double) * S)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.box, sizeof(float) * 4 * P * S)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.status, sizeof(int32_t) * S)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.counters, sizeof(uint32_t) * (2 * (size_t)S + 2))) != OPMM_OK) return rc;
    uint64_t* keys = round_keys;
    if (!keys) {
        if ((rc = ensure(ctx, sc.keys, sizeof(uint64_t) * (size_t)R * S)) != OPMM_OK) return rc;
        keys = (uint64_t*)sc.keys.p;
    }
    FitBufs B;
    B.sacs = (SacDev*)sc.sacs.p;
    B.order = (int*)sc.order.p;
    B.proj = (float*)sc.proj.p;
    B.qorth = (double*)sc.qorth.p;
    B.box = (float*)sc.box.p;
    B.status = (int32_t*)sc.status.p;
    B.counters = (uint32_t*)sc.counters.p;
    B.keys = keys;
    if (prm->screen_rounds > 0 && tiles_per_round > 0) {
        const size_t slots = (size_t)tiles_per_round * kShapes[shape].tpb * kShapes[shape].passes;
        if ((rc = ensure(ctx, sc.costs, sizeof(uint64_t) * slots)) != OPMM_OK) return rc;
        if ((rc = ensure(ctx, sc.tmin, sizeof(uint32_t) * (size_t)tiles_per_round)) != OPMM_OK) return rc;
        if ((rc = ensure(ctx, sc.smin, sizeof(uint64_t) * (size_t)S)) != OPMM_OK) return rc;
        if ((rc = ensure(ctx, sc.vthr, sizeof(double) * (size_t)S)) != OPMM_OK) return rc;
        B.costs = (uint64_t*)sc.costs.p;
        B.tmin = (uint32_t*)sc.tmin.p;
        B.vthr = (double*)sc.vthr.p;
        B.max_T = sc.max_T;
        B.smin = (uint64_t*)sc.smin.p;
    }
    return enqueue_fit_bufs(ctx, B, pos, S, tiles_per_round, prm, shape, seed_opc, opc_out, rmse_out, mae_out,
                            status_out, st, run_prep);
}

// The fit's kernels on given buffers; allocates nothing.
int enqueue_fit_bufs(opmm_ctx* ctx, const FitBufs& B, const float* pos, int S, int tiles_per_round,
                     const opmm_fit_params* prm, int shape, const float* seed_opc, float* opc_out, float* rmse_out,
                     float* mae_out, int32_t* status_out, hipStream_t st, bool run_prep)
{
    const int R = prm->n_rounds;
    uint64_t* keys = B.keys;
    const SacDev* d_sacs = B.sacs;
    float* proj = B.proj;
    double* qorth = B.qorth;
    float* centre = B.box;
    float* hw = centre + P * S;
    float* lo = hw + P * S;
    float* hi = lo + P * S;
    int32_t* status = B.status;
    uint32_t* done = B.counters;
    uint32_t* ready = done + S;
    uint32_t* head = ready + S;
    uint32_t* errflag = head + 1;

    if (run_prep) hipLaunchKernelGGL(prep_kernel, dim3(S), dim3(64), 0, st, S, d_sacs, pos, proj, qorth, status);
    hipLaunchKernelGGL(init_kernel, dim3(blocks_for((int64_t)S * P, 256)), dim3(256), 0, st, S, d_sacs, prm->box_frac,
                       prm->w_init_frac, seed_opc, centre, hw, lo, hi, status);
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for((int64_t)R * S, 256)), dim3(256), 0, st, keys,
                       (int64_t)R * S, ~0ull);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(2 * (int64_t)S + 2, 256)), dim3(256), 0, st, done,
                       2 * (int64_t)S + 2, 0u);
    OPMM_HIP(ctx, hipGetLastError());

    FitLaunch L;
    L.sacs = d_sacs; L.S = S; L.R = R; L.tiles_per_round = tiles_per_round; L.dt = prm->dt_ms;
    L.shrink = prm->shrink; L.proj = proj; L.centre = centre; L.hw = hw; L.lo = lo; L.hi = hi;
    L.status = status; L.keys = keys; L.head = head; L.done = done; L.ready = ready; L.errflag = errflag;
    L.grid_persistent = 0;
    L.ord = B.order;
    L.obase = B.order ? B.order + S : nullptr;
    L.key_stride = S;
    L.wait_limit = ctx->wait_limit;
    L.costs = B.costs;
    L.tmin = B.tmin;
    L.vthr = B.vthr;
    L.max_T = B.max_T;
    L.smin = B.smin;
    L.qorth = qorth;
    L.tau = prm->screen_tol;
    L.timer = nullptr;
    if (ctx->timer.on) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) L.timer = &ctx->timer;
    }
    if (tiles_per_round > 0) {
        if (prm->mode == OPMM_FIT_PERSISTENT) {
            // The queue needs no co-residency, so oversubscribe: blocks that start
            // after the queue has drained exit at once.
            int64_t want = (int64_t)std::max(2, shape_blocks_per_cu(shape)) * 4 * std::max(ctx->cu_count, 1) *
                           256 / kShapes[shape].tpb;
            int64_t total = (int64_t)R * tiles_per_round;
            L.grid_persistent = (int)std::max<int64_t>(1, std::min(want, total));
            OPMM_HIP(ctx, launch_fit_kernel(shape, L, true, 0, st));
            hipLaunchKernelGGL(harvest_giveups_kernel, dim3(1), dim3(64), 0, st, errflag, ctx->giveup_report);
            OPMM_HIP(ctx, hipGetLastError());
        } else {
            for (int r = 0; r < R; ++r) {
                if (r < prm->screen_rounds) {
                    if (!B.costs || !B.tmin || !B.smin || !B.vthr)
                        return fail(ctx, OPMM_EINVAL, "screened rounds need their buffers");
                    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(S, 256)), dim3(256), 0, st, B.smin, (int64_t)S,
                                       ~0ull);
                    OPMM_HIP(ctx, launch_screened_round(shape, L, r, st));
                } else {
                    OPMM_HIP(ctx, launch_fit_kernel(shape, L, false, r, st));
                }
                hipLaunchKernelGGL(refine_kernel, dim3(blocks_for(S, 128)), dim3(128), 0, st, S, d_sacs, r, S, keys,
                                   prm->shrink, centre, hw, lo, hi, status);
                OPMM_HIP(ctx, hipGetLastError());
            }
        }
    }
    hipLaunchKernelGGL(report_kernel, dim3(S), dim3(64), 0, st, S, d_sacs, pos, prm->dt_ms, centre,
                       opc_out, rmse_out, mae_out, status, status_out);
    OPMM_HIP(ctx, hipGetLastError());
    return OPMM_OK;
}

int shape_tile(int shape) { return kShapes[shape].tpb * kShapes[shape].passes; }

// Shapes in the order of a sweep on the full-estimation workload (fastest first).
constexpr int kShapePreference[] = {9, 10, 11, 5, 12, 4, 6, 2, 7, 3, 0, 1, 8};

// The tuned (else default) shape, unless its tile holds more candidates than
// a saccade has: then the fastest shape whose tile fits (empty lanes do no
// work but hold their SIMD slot), else the smallest tile.
int shape_for(const opmm_ctx* ctx, int64_t n_cand)
{
    const int base = ctx->tuned_shape >= 0 ? ctx->tuned_shape : kDefaultShape;
    if (shape_tile(base) <= n_cand) return base;
    int smallest = base;
    for (int sh : kShapePreference) {
        if (shape_tile(sh) <= n_cand) return sh;
        if (shape_tile(sh) < shape_tile(smallest)) smallest = sh;
    }
    return smallest;
}

// Smallest tile: 512 candidates, two per thread.
constexpr int kSmallTileShape = 1;  // tpb256_pass2_unroll1

// Shape for a launch of `tiles` tiles of shape `base`.  A launch with fewer tiles than the device
// has CUs leaves CUs idle, and its time is one block's: the small tile (more, shorter blocks)
// finishes sooner, e.g. one saccade x 4096 candidates in 0.075 instead of 0.125 ms per captured
// fit.  This holds for a shape the autotuner picked too (it times full batches); only an explicit
// opmm_fit_params.tile is kept as given.
int launch_shape_impl(const opmm_ctx* ctx, int base, int64_t tiles)
{
    if (shape_tile(base) <= shape_tile(kSmallTileShape)) return base;
    return tiles < std::max(ctx->cu_count, 1) ? kSmallTileShape : base;
}

int pow2_at_least(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return (int)p;
}

TuneKey tune_key(const opmm_fit_params* prm, const opmm_saccade* sacs, int S)
{
    int max_t = 1;
    int64_t most = 0;
    for (int i = 0; i < S; ++i) {
        max_t = std::max(max_t, (int)sacs[i].T);
        most = std::max<int64_t>(most, sacs[i].n_cand > 0 ? sacs[i].n_cand : prm->n_cand);
    }
    return TuneKey{prm->mode, prm->model, pow2_at_least(max_t), pow2_at_least(std::max(S, 1)), most};
}

int tune_find(const opmm_ctx* ctx, const TuneKey& k)
{
    for (const TuneEntry& e : ctx->tune)
        if (e.key == k) return e.shape;
    return -1;
}

void tune_file(opmm_ctx* ctx, const TuneKey& k, int shape, float ms)
{
    for (TuneEntry& e : ctx->tune)
        if (e.key == k) {
            e.shape = shape;
            e.ms = ms;
            return;
        }
    ctx->tune.push_back(TuneEntry{k, shape, ms});
}

int pick_shape(opmm_ctx* ctx, const opmm_fit_params* prm, const opmm_saccade* sacs, int S)
{
    if (prm->tile >= 0) return prm->tile;
    const int filed = tune_find(ctx, tune_key(prm, sacs, S));
    if (filed >= 0) return filed;
    int64_t most = 0;
    for (int i = 0; i < S; ++i) most = std::max<int64_t>(most, sacs[i].n_cand > 0 ? sacs[i].n_cand : prm->n_cand);
    const int base = shape_for(ctx, most);
    const int64_t tile = shape_tile(base);
    int64_t tiles = 0;
    for (int i = 0; i < S; ++i) tiles += ((sacs[i].n_cand > 0 ? sacs[i].n_cand : prm->n_cand) + tile - 1) / tile;
    return launch_shape_impl(ctx, base, tiles);
}

int check_fit_args(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                   const opmm_fit_params* prm, float* opc_out, float* rmse_out)
{
    if (!ctx) return OPMM_EINVAL;
    int rc;
    if ((rc = validate_params(ctx, prm)) != OPMM_OK) return rc;
    if (S < 0) return fail(ctx, OPMM_EINVAL, "S must be >= 0");
    if (S > 0 && (!pos || !sacs || !opc_out || !rmse_out)) return fail(ctx, OPMM_EINVAL, "NULL array argument");
    if (pos_len < 0) return fail(ctx, OPMM_EINVAL, "pos_len must be >= 0");
    for (int i = 0; i < S; ++i)
        if ((rc = validate_saccade_impl(ctx, sacs[i], pos_len, i)) != OPMM_OK) return rc;
    return OPMM_OK;
}

}  // namespace

namespace opmm_rt {

int validate_saccade(opmm_ctx* ctx, const opmm_saccade& s, int64_t pos_len, int i)
{
    return validate_saccade_impl(ctx, s, pos_len, i);
}

SacDev make_record(const opmm_saccade& s, int n_cand_default)
{
    SacDev d;
    std::memset(&d, 0, sizeof d);
    d.pos_off = s.pos_offset;
    double phi = (double)s.dir_deg * (M_PI / 180.0);
    d.cphi = std::cos(phi);
    d.sphi = std::sin(phi);
    if (s.C == 1) { d.cphi = s.dir_deg == 0.0f ? 1.0 : -1.0; d.sphi = 0.0; }
    d.seed = s.seed;
    d.T = s.T;
    d.C = s.C;
    d.amp = s.amp_deg;
    d.dur = s.dur_ms;
    d.n_cand = s.n_cand > 0 ? s.n_cand : n_cand_default;
    d.tiles = 1;
    d.model = 18;
    return d;
}

hipError_t launch_prep(const SacDev* sacs, int n, const float* pos, const SlotState& ss, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, dim3(n), dim3(64), 0, st, n, sacs, pos, ss.proj, ss.qorth,
                       ss.status);
    return hipGetLastError();
}

hipError_t launch_init(const SacDev* sacs, int n, float box_frac, float w_init_frac, const float* seed_opc,
                       const SlotState& ss, hipStream_t st)
{
    hipLaunchKernelGGL(init_kernel, dim3(blocks_for((int64_t)n * P, 256)), dim3(256), 0, st, n, sacs, box_frac,
                       w_init_frac, seed_opc, ss.centre, ss.hw, ss.lo, ss.hi, ss.status);
    return hipGetLastError();
}

hipError_t launch_reset_keys(const SacDev* sacs, int n, const SlotState& ss, hipStream_t st)
{
    hipLaunchKernelGGL(reset_keys_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, st, n, sacs, ss.keys);
    return hipGetLastError();
}

hipError_t launch_round(int shape, const SacDev* sacs, int n, int tiles_total, float dt, const SlotState& ss,
                        hipStream_t st)
{
    if (tiles_total <= 0) return hipSuccess;
    FitLaunch L;
    std::memset(&L, 0, sizeof L);
    L.sacs = sacs; L.S = n; L.R = 1; L.tiles_per_round = tiles_total; L.key_stride = 0; L.dt = dt;
    L.proj = ss.proj; L.centre = ss.centre; L.hw = ss.hw; L.lo = ss.lo; L.hi = ss.hi;
    L.status = ss.status; L.keys = ss.keys;
    return launch_fit_kernel(shape, L, false, -1, st);
}

hipError_t launch_refine(const SacDev* sacs, int n, float shrink, const SlotState& ss, hipStream_t st)
{
    hipLaunchKernelGGL(refine_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, st, n, sacs, -1, 0, ss.keys, shrink,
                       ss.centre, ss.hw, ss.lo, ss.hi, ss.status);
    return hipGetLastError();
}

hipError_t launch_report(const SacDev* sacs, int n, const float* pos, float dt, const SlotState& ss, float* opc_out,
                         float* rmse_out, float* mae_out, int32_t* status_out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(report_kernel, dim3(n), dim3(64), 0, st, n, sacs, pos, dt, ss.centre, opc_out,
                       rmse_out, mae_out, ss.status, status_out);
    return hipGetLastError();
}

int shape_tile(int shape) { return ::shape_tile(shape); }

int default_shape(const opmm_ctx* ctx) { return ctx->tuned_shape >= 0 ? ctx->tuned_shape : kDefaultShape; }
int shape_for_candidates(const opmm_ctx* ctx, int64_t n_cand) { return ::shape_for(ctx, n_cand); }
int launch_shape(const opmm_ctx* ctx, int base, int64_t tiles) { return launch_shape_impl(ctx, base, tiles); }

int project_batch(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int S,
                  const SacDev** sacs_dev, const float** proj, hipStream_t st)
{
    int rc;
    for (int i = 0; i < S; ++i)
        if ((rc = validate_saccade_impl(ctx, sacs[i], pos_len, i)) != OPMM_OK) return rc;
    FitScratch& sc = ctx->aux;
    int64_t total_T;
    int tiles;
    if ((rc = upload_saccades(ctx, sc, sacs, S, nullptr, 1, &total_T, &tiles, st)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.proj, sizeof(float) * total_T)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.qorth, sizeof(double) * S)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.status, sizeof(int32_t) * S)) != OPMM_OK) return rc;
    if (S > 0) {
        hipLaunchKernelGGL(prep_kernel, dim3(S), dim3(64), 0, st, S, (const SacDev*)sc.sacs.p, pos,
                           (float*)sc.proj.p, (double*)sc.qorth.p, (int32_t*)sc.status.p);
    }
    OPMM_HIP(ctx, hipGetLastError());
    *sacs_dev = (const SacDev*)sc.sacs.p;
    *proj = (const float*)sc.proj.p;
    return OPMM_OK;
}

const int* batch_order(const opmm_ctx* ctx) { return (const int*)ctx->aux.order.p; }

int fit_stage(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int S,
              const opmm_fit_params* prm, float* opc_out, float* rmse_out, FitStage* fs, const SacDev** sacs_dev,
              const float** proj, hipStream_t st)
{
    int rc = check_fit_args(ctx, pos, pos_len, sacs, S, prm, opc_out, rmse_out);
    if (rc != OPMM_OK || S == 0) return rc;
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    FitScratch& sc = ctx->scratch;
    fs->shape = pick_shape(ctx, prm, sacs, S);
    if ((rc = upload_saccades(ctx, sc, sacs, S, prm, shape_tile(fs->shape), &fs->total_T, &fs->tiles, st)) != OPMM_OK)
        return rc;
    if ((rc = ensure(ctx, sc.proj, sizeof(float) * fs->total_T)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.qorth, sizeof(double) * S)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.status, sizeof(int32_t) * S)) != OPMM_OK) return rc;
    hipLaunchKernelGGL(prep_kernel, dim3(S), dim3(64), 0, st, S, (const SacDev*)sc.sacs.p, pos, (float*)sc.proj.p,
                       (double*)sc.qorth.p, (int32_t*)sc.status.p);
    OPMM_HIP(ctx, hipGetLastError());
    *sacs_dev = (const SacDev*)sc.sacs.p;
    *proj = (const float*)sc.proj.p;
    return OPMM_OK;
}

int fit_launch(opmm_ctx* ctx, const float* pos, int S, const FitStage& fs, const opmm_fit_params* prm,
               const float* seed_opc, float* opc_out, float* rmse_out, float* mae_out, int32_t* status_out,
               uint64_t* round_keys, hipStream_t st)
{
    if (S == 0) return OPMM_OK;
    return enqueue_fit(ctx, ctx->scratch, pos, S, fs.total_T, fs.tiles, prm, fs.shape, seed_opc, opc_out, rmse_out,
                       mae_out, status_out, round_keys, st, false);
}

int project_batch_full(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int S,
                       const SacDev** sacs_dev, const float** proj, const double** qorth, const int32_t** status,
                       hipStream_t st)
{
    int rc = project_batch(ctx, pos, pos_len, sacs, S, sacs_dev, proj, st);
    if (rc != OPMM_OK) return rc;
    *qorth = (const double*)ctx->aux.qorth.p;
    *status = (const int32_t*)ctx->aux.status.p;
    return OPMM_OK;
}

}  // namespace opmm_rt

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

void opmm_fit_params_default(opmm_fit_params* p)
{
    if (!p) return;
    p->n_cand = 4096;
    p->n_rounds = 1;
    p->box_frac = 0.25f;
    p->w_init_frac = 1.0f;
    p->shrink = 0.5f;
    p->dt_ms = 1.0f;
    p->mode = OPMM_FIT_ROUNDS;
    p->tile = -1;
    p->model = 18;
    p->screen_rounds = 0;
    p->screen_tol = 5e-5f;
}

void opmm_nominal(float dur_ms, float* out)
{
    if (!out) return;
    for (int j = 0; j < P; ++j) out[j] = nominal_param(j, dur_ms);
}

int opmm_create(opmm_ctx** out, int device)
{
    if (!out) return OPMM_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return OPMM_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return OPMM_EDEVICE;
    opmm_ctx* c = new (std::nothrow) opmm_ctx();
    if (!c) return OPMM_ENOMEM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->cu_count = prop.multiProcessorCount;
        c->arch = prop.gcnArchName;
    }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return OPMM_EDEVICE;
    }
    // The allocation-free fit's scratch: look up this device's copy of the array once, here.
    void* sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) == hipSuccess)
        c->noalloc_scratch = (unsigned char*)sp;
    else
        (void)hipGetLastError();  // opmm_fit_noalloc then reports OPMM_EDEVICE
    if (hipMalloc((void**)&c->giveup_report, sizeof(uint32_t)) != hipSuccess ||
        hipMemset(c->giveup_report, 0, sizeof(uint32_t)) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        opmm_rt::order_init(c->order) != hipSuccess) {
        (void)hipGetLastError();
        if (c->giveup_report) (void)hipFree(c->giveup_report);
        opmm_rt::order_release(c->order);
        (void)hipStreamDestroy(c->cap_stream);
        delete c;
        return OPMM_ENOMEM;
    }
    *out = c;
    return OPMM_OK;
}

int opmm_destroy(opmm_ctx* ctx)
{
    if (!ctx) return OPMM_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->d_cand) (void)hipFree(ctx->d_cand);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->giveup_report) (void)hipFree(ctx->giveup_report);
    opmm_rt::order_release(ctx->order);
    ctx->timer.release();
    delete ctx;
    return OPMM_OK;
}

const char* opmm_last_error(const opmm_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

int opmm_set_wait_limit(opmm_ctx* ctx, uint32_t polls)
{
    if (!ctx) return OPMM_EINVAL;
    ctx->wait_limit = polls;
    return OPMM_OK;
}

int opmm_kernel_timing_enable(opmm_ctx* ctx, int32_t on)
{
    if (!ctx) return OPMM_EINVAL;
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    if (!on) {
        ctx->timer.on = false;
        return OPMM_OK;
    }
    OPMM_HIP(ctx, ctx->timer.reserve());
    ctx->timer.on = true;
    return OPMM_OK;
}

int opmm_kernel_timing_read(opmm_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches)
{
    if (!ctx || !total_ms || !launches || kernel < 0 || kernel >= OPMM_KERNEL_KINDS)
        return fail(ctx, OPMM_EINVAL, "opmm_kernel_timing_read: null handle or output, or unknown kernel");
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    OPMM_HIP(ctx, ctx->timer.collect());
    *total_ms = ctx->timer.ms[kernel];
    *launches = ctx->timer.n[kernel];
    ctx->timer.ms[kernel] = 0.0;
    ctx->timer.n[kernel] = 0;
    return OPMM_OK;
}

int opmm_sync(opmm_ctx* ctx, void* stream)
{
    if (!ctx) return OPMM_EINVAL;
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    OPMM_HIP(ctx, opmm_rt::order_host_wait(ctx->order, (hipStream_t)stream));  // the last call, whatever its stream
    OPMM_HIP(ctx, hipStreamSynchronize((hipStream_t)stream));
    uint32_t n = 0;
    OPMM_HIP(ctx, hipMemcpy(&n, ctx->giveup_report, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (n) OPMM_HIP(ctx, hipMemset(ctx->giveup_report, 0, sizeof(uint32_t)));
    if (n)
        return fail(ctx, OPMM_EDEVICE,
                    std::to_string(n) + " tile(s) of a persistent fit gave up waiting for their round; the "
                    "saccades concerned carry OPMM_ST_WAIT_TIMEOUT and their results are not estimates");
    return OPMM_OK;
}

int opmm_tile_count(void) { return kNumShapes; }
int opmm_tile_default(void) { return kDefaultShape; }

const char* opmm_tile_name(int i) { return (i >= 0 && i < kNumShapes) ? kShapes[i].name : ""; }

int opmm_tune_cache_lookup(opmm_ctx* ctx, const opmm_saccade* sacs, int32_t S, const opmm_fit_params* params,
                           int32_t* tile_out)
{
    if (!ctx) return OPMM_EINVAL;
    if (!params || !tile_out || S < 0 || (S > 0 && !sacs)) return fail(ctx, OPMM_EINVAL, "bad arguments");
    *tile_out = tune_find(ctx, tune_key(params, sacs, S));
    return OPMM_OK;
}

int opmm_tune_cache_save(opmm_ctx* ctx, const char* path)
{
    if (!ctx) return OPMM_EINVAL;
    if (!path) return fail(ctx, OPMM_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(ctx, OPMM_EINVAL, std::string("cannot write ") + path);
    bool ok = std::fprintf(f, "# opmm autotuner cache: arch mode model t_bucket s_bucket n_cand shape ms\n") > 0;
    for (const TuneEntry& e : ctx->tune)
        ok = ok && std::fprintf(f, "%s %d %d %d %d %lld %s %.4f\n", ctx->arch.c_str(), e.key.mode, e.key.model,
                                e.key.t_bucket, e.key.s_bucket, (long long)e.key.n_cand, kShapes[e.shape].name,
                                (double)e.ms) > 0;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? OPMM_OK : fail(ctx, OPMM_EINVAL, std::string("write failed: ") + path);
}

int opmm_tune_cache_load(opmm_ctx* ctx, const char* path)
{
    if (!ctx) return OPMM_EINVAL;
    if (!path) return fail(ctx, OPMM_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(ctx, OPMM_EINVAL, std::string("cannot read ") + path);
    std::vector<TuneEntry> add;
    char line[512];
    int lineno = 0, rc = OPMM_OK;
    while (rc == OPMM_OK && std::fgets(line, sizeof line, f)) {
        ++lineno;
        if (line[0] == '#' || line[0] == '\n' || line[0] == '\0') continue;
        char arch[256], name[128];
        int mode, model, tb, sb;
        long long nc;
        float ms;
        if (std::sscanf(line, "%255s %d %d %d %d %lld %127s %f", arch, &mode, &model, &tb, &sb, &nc, name, &ms) != 8 ||
            (mode != OPMM_FIT_ROUNDS && mode != OPMM_FIT_PERSISTENT) || (model != 18 && model != 9) || tb < 1 ||
            sb < 1 || nc < 1) {
            rc = fail(ctx, OPMM_EINVAL, std::string("malformed autotuner cache line ") + std::to_string(lineno) +
                                            " in " + path);
            break;
        }
        if (ctx->arch != arch) continue;  // written for another device
        int shape = -1;
        for (int i = 0; i < kNumShapes; ++i)
            if (std::strcmp(kShapes[i].name, name) == 0) shape = i;
        if (shape < 0) continue;  // a shape this build does not have
        add.push_back(TuneEntry{TuneKey{mode, model, tb, sb, (int64_t)nc}, shape, ms});
    }
    std::fclose(f);
    if (rc != OPMM_OK) return rc;
    for (const TuneEntry& e : add) tune_file(ctx, e.key, e.shape, e.ms);
    return OPMM_OK;
}

int opmm_candidates(opmm_ctx* ctx, uint64_t seed, uint32_t round, uint32_t idx0, int64_t n, const float* c,
                    const float* w, const float* lo, const float* hi, float* out, void* stream)
{
    if (!ctx) return OPMM_EINVAL;
    if (n < 0 || (n > 0 && (!c || !w || !lo || !hi || !out))) return fail(ctx, OPMM_EINVAL, "bad arguments");
    if ((uint64_t)idx0 + (uint64_t)n > 0x100000000ull) return fail(ctx, OPMM_EINVAL, "index beyond 2^32");
    if (round >= (1u << 28)) return fail(ctx, OPMM_EINVAL, "round beyond 2^28");
    if (n == 0) return OPMM_OK;
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    BoxArg ba;
    std::memcpy(ba.v[0], c, sizeof(float) * P);
    std::memcpy(ba.v[1], w, sizeof(float) * P);
    std::memcpy(ba.v[2], lo, sizeof(float) * P);
    std::memcpy(ba.v[3], hi, sizeof(float) * P);
    hipLaunchKernelGGL(candidates_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, seed, round,
                       idx0, n, ba, out);
    OPMM_HIP(ctx, hipGetLastError());
    return OPMM_OK;
}

int opmm_simulate(opmm_ctx* ctx, const float* opc, const float* amp, int64_t n, int32_t T, float dt_ms,
                  float* traj_out, void* stream)
{
    if (!ctx) return OPMM_EINVAL;
    if (n < 0) return fail(ctx, OPMM_EINVAL, "n must be >= 0");
    if (T < 1 || T > OPMM_MAX_T) return fail(ctx, OPMM_EINVAL, "T out of range");
    if (!(dt_ms > 0.0f && dt_ms <= 1.0f)) return fail(ctx, OPMM_EINVAL, "dt_ms must be in (0, 1]");
    if (n > 0 && (!opc || !amp || !traj_out)) return fail(ctx, OPMM_EINVAL, "NULL array argument");
    if (n == 0) return OPMM_OK;
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(simulate_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, n, opc, amp, T,
                       dt_ms, traj_out);
    OPMM_HIP(ctx, hipGetLastError());
    return OPMM_OK;
}

namespace {

int score_impl(opmm_ctx* ctx, const float* opc, int64_t n, const float* pos, int64_t pos_len, const opmm_saccade* sac,
               float dt_ms, float* rmse_out, void* stream, bool fp32)
{
    if (!ctx) return OPMM_EINVAL;
    if (!sac) return fail(ctx, OPMM_EINVAL, "sac is NULL");
    int rc;
    if ((rc = validate_saccade_impl(ctx, *sac, pos_len, 0)) != OPMM_OK) return rc;
    if (!(dt_ms > 0.0f && dt_ms <= 1.0f)) return fail(ctx, OPMM_EINVAL, "dt_ms must be in (0, 1]");
    if (n < 0) return fail(ctx, OPMM_EINVAL, "n must be >= 0");
    if (n > 0 && (!opc || !pos || !rmse_out)) return fail(ctx, OPMM_EINVAL, "NULL array argument");
    if (n == 0) return OPMM_OK;
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    opmm_rt::Ordered ord(ctx->order, st);
    OPMM_HIP(ctx, ord.error());
    FitScratch& sc = ctx->scratch;
    int64_t total_T;
    int tiles;
    if ((rc = upload_saccades(ctx, sc, sac, 1, nullptr, 1, &total_T, &tiles, st)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.proj, sizeof(float) * total_T)) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.qorth, sizeof(double))) != OPMM_OK) return rc;
    if ((rc = ensure(ctx, sc.status, sizeof(int32_t))) != OPMM_OK) return rc;
    hipLaunchKernelGGL(prep_kernel, dim3(1), dim3(64), 0, st, 1, (const SacDev*)sc.sacs.p, pos, (float*)sc.proj.p,
                       (double*)sc.qorth.p, (int32_t*)sc.status.p);
    if (fp32)
        hipLaunchKernelGGL(score_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, opc,
                           (const float*)sc.proj.p, sac->T, sac->C, (const double*)sc.qorth.p, sac->amp_deg, dt_ms,
                           rmse_out);
    else
        hipLaunchKernelGGL(score_kernel<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, opc,
                           (const float*)sc.proj.p, sac->T, sac->C, (const double*)sc.qorth.p, sac->amp_deg, dt_ms,
                           rmse_out);
    OPMM_HIP(ctx, hipGetLastError());
    return OPMM_OK;
}

}  // namespace

int opmm_score(opmm_ctx* ctx, const float* opc, int64_t n, const float* pos, int64_t pos_len,
               const opmm_saccade* sac, float dt_ms, float* rmse_out, void* stream)
{
    return score_impl(ctx, opc, n, pos, pos_len, sac, dt_ms, rmse_out, stream, false);
}

int opmm_score_screen(opmm_ctx* ctx, const float* opc, int64_t n, const float* pos, int64_t pos_len,
                      const opmm_saccade* sac, float dt_ms, float* rmse_out, void* stream)
{
    return score_impl(ctx, opc, n, pos, pos_len, sac, dt_ms, rmse_out, stream, true);
}

int opmm_fit(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
             const opmm_fit_params* params, const float* seed_opc, float* opc_out, float* rmse_out, float* mae_out,
             int32_t* status_out, uint64_t* round_keys, void* stream)
{
    if (!ctx) return OPMM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    opmm_rt::Ordered ord(ctx->order, st);
    OPMM_HIP(ctx, ord.error());
    opmm_rt::FitStage fs;
    const SacDev* sd;
    const float* proj;
    int rc = opmm_rt::fit_stage(ctx, pos, pos_len, sacs, S, params, opc_out, rmse_out, &fs, &sd, &proj, st);
    if (rc != OPMM_OK || S == 0) return rc;
    return opmm_rt::fit_launch(ctx, pos, S, fs, params, seed_opc, opc_out, rmse_out, mae_out, status_out, round_keys,
                               st);
}

int opmm_fit_plan_create(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                         const opmm_fit_params* params, const float* seed_opc, float* opc_out, float* rmse_out,
                         float* mae_out, int32_t* status_out, uint64_t* round_keys, void* stream, opmm_plan** out)
{
    if (!out) return fail(ctx, OPMM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_fit_args(ctx, pos, pos_len, sacs, S, params, opc_out, rmse_out);
    if (rc != OPMM_OK) return rc;
    if (S == 0) return fail(ctx, OPMM_EINVAL, "a plan needs S >= 1");
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    opmm_plan* pl = new (std::nothrow) opmm_plan();
    if (!pl) return fail(ctx, OPMM_ENOMEM, "plan allocation failed");
    pl->ctx = ctx;
    if (opmm_rt::order_init(pl->order) != hipSuccess) {
        (void)hipGetLastError();
        delete pl;
        return fail(ctx, OPMM_EDEVICE, "plan event creation failed");
    }
    const int shape = pick_shape(ctx, params, sacs, S);
    int64_t total_T;
    int tiles;
    hipStream_t cs = ctx->cap_stream;
    rc = upload_saccades(ctx, pl->scratch, sacs, S, params, shape_tile(shape), &total_T, &tiles, cs);
    if (rc == OPMM_OK) {
        // allocate outside the capture: enqueue once for real, then capture
        rc = enqueue_fit(ctx, pl->scratch, pos, S, total_T, tiles, params, shape, seed_opc, opc_out, rmse_out,
                         mae_out, status_out, round_keys, cs);
    }
    if (rc == OPMM_OK && hipStreamSynchronize(cs) != hipSuccess) rc = fail(ctx, OPMM_EDEVICE, "plan warm-up failed");
    if (rc == OPMM_OK) {
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) rc = hip_fail(ctx, e, "hipStreamBeginCapture");
        else {
            rc = enqueue_fit(ctx, pl->scratch, pos, S, total_T, tiles, params, shape, seed_opc, opc_out, rmse_out,
                             mae_out, status_out, round_keys, cs);
            hipError_t e2 = hipStreamEndCapture(cs, &pl->graph);
            if (rc == OPMM_OK && e2 != hipSuccess) rc = hip_fail(ctx, e2, "hipStreamEndCapture");
        }
    }
    if (rc == OPMM_OK) {
        hipError_t e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail(ctx, e, "hipGraphInstantiate");
    }
    (void)stream;
    if (rc != OPMM_OK) {
        opmm_plan_destroy(pl);
        return rc;
    }
    *out = pl;
    return OPMM_OK;
}

int opmm_plan_launch(opmm_plan* plan, void* stream)
{
    if (!plan || !plan->exec) return OPMM_EINVAL;
    opmm_ctx* ctx = plan->ctx;
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    opmm_rt::Ordered ord(plan->order, (hipStream_t)stream);  // launches of one plan share its scratch
    OPMM_HIP(ctx, ord.error());
    OPMM_HIP(ctx, hipGraphLaunch(plan->exec, (hipStream_t)stream));
    return OPMM_OK;
}

int opmm_plan_destroy(opmm_plan* plan)
{
    if (!plan) return OPMM_OK;
    (void)hipSetDevice(plan->ctx->device);
    (void)hipDeviceSynchronize();
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    opmm_rt::order_release(plan->order);
    delete plan;
    return OPMM_OK;
}

int opmm_autotune(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                  const opmm_fit_params* params, int32_t* tile_out, void* stream)
{
    int rc = check_fit_args(ctx, pos, pos_len, sacs, S, params, (float*)1, (float*)1);
    if (rc != OPMM_OK) return rc;
    if (S == 0) return fail(ctx, OPMM_EINVAL, "autotune needs S >= 1");
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    opmm_rt::Ordered ord(ctx->order, st);
    OPMM_HIP(ctx, ord.error());
    // sample: every k-th saccade, at most 256
    const int stride = std::max(1, S / 256);
    std::vector<opmm_saccade> sub;
    for (int i = 0; i < S; i += stride) sub.push_back(sacs[i]);
    const int Ss = (int)sub.size();
    // the caller's mode; enough rounds that the sample sees both the wide early boxes (many
    // distinct pulse ends per tile) and the narrow later ones
    opmm_fit_params pp = *params;
    pp.n_rounds = std::min(params->n_rounds, 4);
    DevBuf out;
    if ((rc = ensure(ctx, out, sizeof(float) * (size_t)Ss * (P + 1))) != OPMM_OK) return rc;
    float* d_opc = (float*)out.p;
    float* d_rmse = d_opc + (size_t)Ss * P;
    hipEvent_t e0, e1;
    OPMM_HIP(ctx, hipEventCreate(&e0));
    OPMM_HIP(ctx, hipEventCreate(&e1));
    int best = 0;
    float best_ms = 1e30f;
    for (int sh = 0; sh < kNumShapes && rc == OPMM_OK; ++sh) {
        pp.tile = sh;
        float ms_best = 1e30f;
        for (int rep = 0; rep < 3 && rc == OPMM_OK; ++rep) {
            (void)hipEventRecord(e0, st);
            rc = opmm_fit(ctx, pos, pos_len, sub.data(), Ss, &pp, nullptr, d_opc, d_rmse, nullptr, nullptr, nullptr,
                          stream);
            (void)hipEventRecord(e1, st);
            if (rc == OPMM_OK && hipEventSynchronize(e1) == hipSuccess) {
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) ms_best = std::min(ms_best, ms);
            }
        }
        if (ms_best < best_ms) {
            best_ms = ms_best;
            best = sh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipDeviceSynchronize();
    (void)hipFree(out.p);
    if (rc != OPMM_OK) return rc;
    ctx->tuned_shape = best;
    tune_file(ctx, tune_key(params, sacs, S), best, best_ms);
    if (tile_out) *tile_out = best;
    return OPMM_OK;
}

// Host staging of opmm_fit_noalloc: static, shared by every call and guarded
// by its mutex until the records are on the device.
namespace {
struct NoallocStage {
    std::mutex mu;
    SacDev recs[OPMM_NOALLOC_MAX_S];
    int order[2 * OPMM_NOALLOC_MAX_S];
    int cnt[OPMM_MAX_T + 1];
};
NoallocStage g_noalloc_stage;
}  // namespace

int opmm_fit_noalloc(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                     const opmm_fit_params* params, const float* seed_opc, float* opc_out, float* rmse_out,
                     float* mae_out, int32_t* status_out, uint64_t* round_keys, void* stream)
{
    int rc = check_fit_args(ctx, pos, pos_len, sacs, S, params, opc_out, rmse_out);
    if (rc != OPMM_OK || S == 0) return rc;
    if (S > OPMM_NOALLOC_MAX_S) return fail(ctx, OPMM_EINVAL, "S exceeds OPMM_NOALLOC_MAX_S");
    if (params->screen_rounds > 0)
        return fail(ctx, OPMM_EINVAL, "the allocation-free fit runs every round in FP64 (screen_rounds = 0)");
    if (!ctx->noalloc_scratch) return fail(ctx, OPMM_EDEVICE, "no device address for the allocation-free scratch");
    OPMM_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    opmm_rt::Ordered ord(ctx->order, st);
    OPMM_HIP(ctx, ord.error());
    const int shape = pick_shape(ctx, params, sacs, S);
    NoallocStage& g = g_noalloc_stage;
    std::lock_guard<std::mutex> lock(g.mu);
    int64_t total_T, tiles;
    build_records(sacs, S, params, shape_tile(shape), g.recs, g.order, g.cnt, &total_T, &tiles);
    if (tiles > 0x7FFFFFFF / 8) return fail(ctx, OPMM_EINVAL, "too many candidate tiles in one batch");
    // carve the scratch: each part 256-byte aligned
    size_t off = 0;
    auto carve = [&off](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_sacs = carve(sizeof(SacDev) * (size_t)S), o_ord = carve(sizeof(int) * 2 * (size_t)S),
                 o_proj = carve(sizeof(float) * (size_t)total_T), o_q = carve(sizeof(double) * (size_t)S),
                 o_box = carve(sizeof(float) * 4 * P * (size_t)S), o_st = carve(sizeof(int32_t) * (size_t)S),
                 o_cnt = carve(sizeof(uint32_t) * (2 * (size_t)S + 2)),
                 o_keys = round_keys ? 0 : carve(sizeof(uint64_t) * (size_t)params->n_rounds * S);
    if (off > (size_t)OPMM_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, OPMM_EINVAL, "the batch needs " + std::to_string(off) + " bytes of scratch; the "
                    "allocation-free fit has " + std::to_string((size_t)OPMM_NOALLOC_SCRATCH_BYTES));
    unsigned char* base = ctx->noalloc_scratch;
    FitBufs B;
    B.sacs = (SacDev*)(base + o_sacs);
    B.order = (int*)(base + o_ord);
    B.proj = (float*)(base + o_proj);
    B.qorth = (double*)(base + o_q);
    B.box = (float*)(base + o_box);
    B.status = (int32_t*)(base + o_st);
    B.counters = (uint32_t*)(base + o_cnt);
    B.keys = round_keys ? round_keys : (uint64_t*)(base + o_keys);
    OPMM_HIP(ctx, hipMemcpyAsync(B.sacs, g.recs, sizeof(SacDev) * (size_t)S, hipMemcpyHostToDevice, st));
    OPMM_HIP(ctx, hipMemcpyAsync(B.order, g.order, sizeof(int) * 2 * (size_t)S, hipMemcpyHostToDevice, st));
    OPMM_HIP(ctx, hipStreamSynchronize(st));
    // every part is written before it is read: records and order above, projection, energies and
    // status by the prep kernel, the box by init, counters and keys by fill kernels
    return enqueue_fit_bufs(ctx, B, pos, S, (int)tiles, params, shape, seed_opc, opc_out, rmse_out, mae_out,
                            status_out, st, true);
}

}  // extern "C"
