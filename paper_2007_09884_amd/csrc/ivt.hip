// libopmm: saccade extraction from a raw gaze stream by velocity threshold
// (I-VT, Salvucci & Goldberg 2000), the identification step the paper runs
// before estimation (Section 3.1: recorded, cleaned, saccades extracted;
// Section 4: I-VT, saccades shorter than 6 ms discarded).
//
// A sample k >= 1 is a saccade sample when its point-to-point speed
// |g_k - g_{k-1}| / dt exceeds the threshold; a saccade is a maximal run of
// saccade samples, its trace the run with the sample before it (the last
// fixation sample) prepended, re-based to that sample.  Runs with duration
// (T - 1) * dt below min_dur_ms or amplitude below min_amp_deg are dropped.
// Output order is the stream order: segment starts are compacted with block
// counts and a scan, never with an unordered atomic append.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/opmm.h"
#include "runtime.hpp"

namespace {

constexpr int IVT_TPB = 256;

__device__ __forceinline__ bool fast(const float* g, int64_t k, float thr2)
{
    const float dx = g[2 * k] - g[2 * k - 2], dy = g[2 * k + 1] - g[2 * k - 1];
    return dx * dx + dy * dy > thr2;
}

// flag[k] = 1 if a run of fast samples starts at k; per-block start counts
__global__ void ivt_starts_kernel(const float* __restrict__ g, int64_t N, float thr2, int32_t* __restrict__ blk)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * IVT_TPB + threadIdx.x;
    if (k >= 1 && k < N && fast(g, k, thr2) && (k == 1 || !fast(g, k - 1, thr2))) atomicAdd(&cnt, 1);
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = cnt;
}

// exclusive scan of n ints in place by one block (n up to millions: serial chunks)
__global__ void scan_kernel(int32_t* a, int64_t n, int32_t* total)
{
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t b = t * per, e = min(n, b + per);
    int32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += a[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int32_t run = 0;
        for (int i = 0; i < 1024; ++i) { int32_t v = part[i]; part[i] = run; run += v; }
        *total = run;
    }
    __syncthreads();
    int32_t run = part[t];
    for (int64_t i = b; i < e; ++i) { int32_t v = a[i]; a[i] = run; run += v; }
}

// write the start sample of every run, in stream order
__global__ void ivt_scatter_kernel(const float* __restrict__ g, int64_t N, float thr2, const int32_t* __restrict__ blk,
                                   int64_t* __restrict__ starts)
{
    __shared__ int32_t pre[IVT_TPB];
    const int64_t k = (int64_t)blockIdx.x * IVT_TPB + threadIdx.x;
    const int f = (k >= 1 && k < N && fast(g, k, thr2) && (k == 1 || !fast(g, k - 1, thr2))) ? 1 : 0;
    pre[threadIdx.x] = f;
    __syncthreads();
    for (int o = 1; o < IVT_TPB; o <<= 1) {  // inclusive block scan
        int32_t v = threadIdx.x >= o ? pre[threadIdx.x - o] : 0;
        __syncthreads();
        pre[threadIdx.x] += v;
        __syncthreads();
    }
    if (f) starts[blk[blockIdx.x] + pre[threadIdx.x] - 1] = k;
}

// per run: length, amplitude, direction, acceptance
__global__ void ivt_segments_kernel(const float* __restrict__ g, int64_t N, float thr2, int32_t n_runs,
                                    const int64_t* __restrict__ starts, float dt, float min_dur, float min_amp,
                                    int32_t max_T, int32_t* __restrict__ keep, int32_t* __restrict__ Ts,
                                    float* __restrict__ amp, float* __restrict__ dir)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_runs) return;
    const int64_t k0 = starts[i];
    int64_t k1 = k0;
    while (k1 + 1 < N && fast(g, k1 + 1, thr2)) ++k1;
    const int64_t T = k1 - k0 + 2;  // the fixation sample before the run + the run
    const float dx = g[2 * k1] - g[2 * (k0 - 1)], dy = g[2 * k1 + 1] - g[2 * (k0 - 1) + 1];
    const float a = sqrtf(dx * dx + dy * dy);
    float d = atan2f(dy, dx) * (180.0f / 3.14159265358979f);
    if (d < 0.0f) d += 360.0f;
    Ts[i] = (int32_t)min(T, (int64_t)0x7FFFFFFF);
    amp[i] = a;
    dir[i] = d;
    keep[i] = ((float)(T - 1) * dt >= min_dur && a >= min_amp && T <= max_T) ? 1 : 0;
}

// kept runs -> records and traces re-based to their first sample
__global__ void ivt_emit_kernel(const float* __restrict__ g, int32_t n_runs, const int64_t* __restrict__ starts,
                                const int32_t* __restrict__ keep, const int32_t* __restrict__ slot,
                                const int32_t* __restrict__ off, const int32_t* __restrict__ Ts,
                                const float* __restrict__ amp, const float* __restrict__ dir, float dt,
                                uint64_t seed_base, int32_t max_out, opmm_saccade* __restrict__ out,
                                float* __restrict__ out_pos, int64_t* __restrict__ src_start)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_runs || !keep[i]) return;
    const int o = slot[i];
    if (o >= max_out) return;
    const int64_t k = starts[i] - 1;
    const int T = Ts[i];
    const int64_t po = 2 * (int64_t)off[i];
    const float x0 = g[2 * k], y0 = g[2 * k + 1];
    for (int t = 0; t < T; ++t) {
        out_pos[po + 2 * t] = g[2 * (k + t)] - x0;
        out_pos[po + 2 * t + 1] = g[2 * (k + t) + 1] - y0;
    }
    opmm_saccade s;
    s.pos_offset = po;
    s.T = T;
    s.C = 2;
    s.amp_deg = amp[i];
    s.dir_deg = dir[i];
    s.dur_ms = (float)(T - 1) * dt;
    s.n_cand = 0;
    s.seed = seed_base + (uint64_t)k;
    out[o] = s;
    if (src_start) src_start[o] = k;
}

int blocks_of(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

extern "C" {

int opmm_ivt_extract(opmm_ctx* ctx, const float* gaze, int64_t N, float dt_ms, float vel_thresh_deg_s,
                     float min_dur_ms, float min_amp_deg, int32_t max_T, uint64_t seed_base, int32_t max_out,
                     opmm_saccade* sacs_out, float* pos_out, int64_t pos_cap, int64_t* src_start_out,
                     int32_t* n_out, void* stream)
{
    if (!ctx || !n_out) return OPMM_EINVAL;
    *n_out = 0;
    if (N < 0 || (N > 0 && !gaze) || !(dt_ms > 0) || !(vel_thresh_deg_s >= 0) || !(min_dur_ms >= 0) ||
        !(min_amp_deg >= 0) || max_T < 2 || max_T > OPMM_MAX_T || max_out < 0 ||
        (max_out > 0 && (!sacs_out || !pos_out)))
        return opmm_rt::fail(ctx, OPMM_EINVAL, "bad I-VT arguments");
    if (N < 2 || max_out == 0) return OPMM_OK;
    hipStream_t st = (hipStream_t)stream;
    const float v_per_sample = vel_thresh_deg_s * dt_ms * 1e-3f;  // deg per sample at the threshold
    const float thr2 = v_per_sample * v_per_sample;
    const int nb = blocks_of(N, IVT_TPB);
    int32_t *blk = nullptr, *tot = nullptr;
    int64_t* starts = nullptr;
    int rc = OPMM_OK;
    auto ok = [&](hipError_t e, const char* w) { if (rc == OPMM_OK && e != hipSuccess) rc = opmm_rt::hip_fail(ctx, e, w); };
    ok(hipMallocAsync((void**)&blk, sizeof(int32_t) * (nb + 1), st), "alloc");
    ok(hipMallocAsync((void**)&tot, sizeof(int32_t) * 2, st), "alloc");
    int32_t n_runs = 0;
    if (rc == OPMM_OK) {
        hipLaunchKernelGGL(ivt_starts_kernel, dim3(nb), dim3(IVT_TPB), 0, st, gaze, N, thr2, blk);
        hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, blk, (int64_t)nb, tot);
        ok(hipMemcpyAsync(&n_runs, tot, sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy");
        ok(hipStreamSynchronize(st), "sync");
    }
    if (rc == OPMM_OK && n_runs > 0) {
        // one allocation for the per-run arrays: starts (int64), then seven 4-byte arrays: keep, T,
        // slot, offset, keep after truncation (int32), amplitude, direction (float).  keep and T are
        // adjacent (one copy down), and so are slot, offset and the truncated keep (one copy up).
        const size_t R = (size_t)n_runs;
        char* runbuf = nullptr;
        ok(hipMallocAsync((void**)&runbuf, R * (sizeof(int64_t) + 7 * sizeof(int32_t)), st), "alloc");
        if (rc != OPMM_OK) runbuf = nullptr;
        starts = (int64_t*)runbuf;
        if (rc == OPMM_OK) {
            int32_t* keep = (int32_t*)(runbuf + R * sizeof(int64_t));
            int32_t* Ts = keep + R;
            int32_t* slot = Ts + R;
            int32_t* off = slot + R;
            int32_t* keep2 = off + R;  // keep after truncation
            float* amp = (float*)(keep2 + R);
            float* dir = amp + R;
            hipLaunchKernelGGL(ivt_scatter_kernel, dim3(nb), dim3(IVT_TPB), 0, st, gaze, N, thr2, blk, starts);
            hipLaunchKernelGGL(ivt_segments_kernel, dim3(blocks_of(n_runs, 128)), dim3(128), 0, st, gaze, N, thr2,
                               n_runs, starts, dt_ms, min_dur_ms, min_amp_deg, max_T, keep, Ts, amp, dir);
            std::vector<int32_t> hkT(2 * R);  // keep, then T
            ok(hipMemcpyAsync(hkT.data(), keep, sizeof(int32_t) * 2 * R, hipMemcpyDeviceToHost, st), "copy");
            ok(hipStreamSynchronize(st), "sync");
            if (rc == OPMM_OK) {
                // output slot and trace offset of the kept runs, in stream order; output stops at the
                // first kept run past max_out records or pos_cap floats of trace (a prefix of the stream)
                const int32_t* hk = hkT.data();
                const int32_t* hT = hk + R;
                std::vector<int32_t> up(3 * R, 0);  // slot, offset, keep after truncation
                int32_t* hs = up.data();
                int32_t* ho = hs + R;
                int32_t* hk2 = ho + R;
                int64_t acc = 0;
                int32_t emitted = 0;
                bool full = false;
                for (size_t i = 0; i < R; ++i) {
                    if (!hk[i]) continue;
                    full = full || emitted >= max_out || 2 * (acc + hT[i]) > pos_cap;
                    if (full) continue;
                    hk2[i] = 1;
                    ho[i] = (int32_t)acc;
                    hs[i] = emitted;
                    acc += hT[i];
                    ++emitted;
                }
                opmm_saccade* d_recs = nullptr;
                int64_t* d_src = nullptr;
                ok(hipMallocAsync((void**)&d_recs, sizeof(opmm_saccade) * std::max(emitted, 1), st), "alloc");
                ok(hipMallocAsync((void**)&d_src, sizeof(int64_t) * std::max(emitted, 1), st), "alloc");
                ok(hipMemcpyAsync(slot, up.data(), sizeof(int32_t) * 3 * R, hipMemcpyHostToDevice, st), "copy");
                if (rc == OPMM_OK)
                    hipLaunchKernelGGL(ivt_emit_kernel, dim3(blocks_of(n_runs, 128)), dim3(128), 0, st, gaze, n_runs,
                                       starts, keep2, slot, off, Ts, amp, dir, dt_ms, seed_base, max_out, d_recs,
                                       pos_out, d_src);
                if (emitted > 0) {
                    ok(hipMemcpyAsync(sacs_out, d_recs, sizeof(opmm_saccade) * emitted, hipMemcpyDeviceToHost, st),
                       "copy");
                    if (src_start_out)
                        ok(hipMemcpyAsync(src_start_out, d_src, sizeof(int64_t) * emitted, hipMemcpyDeviceToHost, st),
                           "copy");
                }
                ok(hipStreamSynchronize(st), "sync");
                if (d_recs) (void)hipFreeAsync(d_recs, st);
                if (d_src) (void)hipFreeAsync(d_src, st);
                *n_out = emitted;
            }
        }
    }
    if (starts) (void)hipFreeAsync(starts, st);
    if (blk) (void)hipFreeAsync(blk, st);
    if (tot) (void)hipFreeAsync(tot, st);
    return rc;
}

}  // extern "C"
