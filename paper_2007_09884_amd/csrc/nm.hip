// libopmm: the paper's own estimator -- a parallel Nelder-Mead per saccade
// (Section 3.3, Algorithm 1): one task per saccade, all simplex transforms of
// an iteration evaluated simultaneously, the simplex sorted every iteration,
// both exit tolerances or an iteration cap.
//
// One or two saccades per 64-lane wave.  The simplex (19 vertices x 18
// coordinates, FP64, relative to the Table 1 nominal) and the projected trace
// (sized to the batch's longest) live in LDS.  Every iteration lanes 0..21 of
// a task build and evaluate reflection, expansion, outside and inside
// contraction and the 18 shrink vertices at once; lane 0 of the task takes the
// Lagarias decision (reflection 1, expansion 2, contraction 1/2, shrink 1/2);
// the exit test, the vertex update and the stable re-sort run one coordinate
// or one vertex per lane.  Each evaluation is the same plant
// simulation and RMSE as the box search (points clamped to the search box and
// rounded to FP32, the candidate format).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/opmm.h"
#include "plant.hpp"
#include "runtime.hpp"

using namespace opmm;
using opmm_rt::SacDev;

namespace {

constexpr int NV = P + 1;   // simplex vertices
constexpr int NPT = 4 + P;  // points per iteration: r, e, oc, ic, 18 shrink

// One task's simplex state (the trace lives in dynamic LDS after the groups).
struct NmGroup {
    double v[NV][P];
    double f[NV];
    double pt[NPT][P];
    double fp[NPT];
    double xb[P];
    double nom[P];
    double tv[NV][P];  // sort staging
    double tf[NV];
    double dxc[P];     // per-coordinate spread of the simplex
    int flag;          // exit test passed
    int dec;
    int active;        // still iterating
    int iters;         // iterations taken (set when the task stops)
};

struct SseSinkNm {
    const R* r;
    double sse;
    __device__ __forceinline__ void operator()(int k, R dth, R theq)
    {
        R e = (r[k] - theq) - dth;
        sse = fma((double)e, (double)e, sse);
    }
};

// RMSE of point x (relative to nominal) for this lane; all 64 lanes call it
// (wave-uniform bounds), `valid` lanes' results are meaningful.
__device__ double nm_eval(const NmGroup& g, const R* r, const double* x, bool valid, const SacDev& sd, double q,
                          float dt, double lo, double hi)
{
    float p[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double v = valid ? x[j] : 1.0;
        v = fmin(fmax(v, lo), hi);
        p[j] = (float)(v * g.nom[j]);
    }
    Plant pl;
    plant_setup(p, sd.amp, dt, pl);
    R frac;
    int k0 = pulse_end_sample(pl.pwd, sd.T, frac);
    int kmin = __builtin_amdgcn_readfirstlane(wave_min(valid ? k0 : 0x7FFFFFFF));
    int kmax = __builtin_amdgcn_readfirstlane(wave_max(valid ? k0 : -0x7FFFFFFF));
    SseSinkNm sink{r, 0.0};
    if (valid) run_trajectory<2>(pl, sd.T, (R)dt, k0, frac, kmin, kmax, sink);
    double rm = sqrt((sink.sse + q) / ((double)sd.T * sd.C));
    return (rm >= 0.0 && rm <= 1.7976931348623157e308) ? rm : INFINITY;
}

// Stable sort of a simplex by value, in parallel: vertex i goes to rank
// #{k : f_k < f_i} + #{k < i : f_k == f_i} (the order a stable insertion sort
// gives), each lane of the group moves one row.  Every lane of the wave calls it.
__device__ void nm_sort(NmGroup& g, int l, bool on)
{
    if (on && l < NV) {
        const double fi = g.f[l];
        int rank = 0;
        for (int k = 0; k < NV; ++k) rank += (g.f[k] < fi) || (k < l && g.f[k] == fi);
        for (int j = 0; j < P; ++j) g.tv[rank][j] = g.v[l][j];
        g.tf[rank] = fi;
    }
    __syncthreads();
    if (on && l < NV) {
        for (int j = 0; j < P; ++j) g.v[l][j] = g.tv[l][j];
        g.f[l] = g.tf[l];
    }
    __syncthreads();
}

// G tasks per 64-lane wave (1 or 2): lanes 64/G * g .. of group g work on saccade G * block + g, 22
// of them evaluating.  Every group runs the same instruction stream; a finished group's lanes idle
// until the other one ends.  deadline_ticks > 0: a task still iterating when that many ticks of the
// wall clock (wall_clock64) have passed since the launch started ends there with OPMM_ST_DEADLINE.
template <int G>
__global__ __launch_bounds__(64) void nm_kernel(int S, const SacDev* __restrict__ sacs, const float* __restrict__ proj,
                                                const double* __restrict__ qorth, const int32_t* __restrict__ status_in,
                                                const float* __restrict__ seed_opc, int max_iter, double tol_x,
                                                double tol_f, double lo, double hi, float dt, int max_T,
                                                uint64_t deadline_ticks, float* opc_out, float* rmse_out,
                                                int32_t* iters_out, int8_t* dec_out, int32_t* status_out)
{
    constexpr int LG = 64 / G;
    __shared__ NmGroup gs[G];
    __shared__ int s_stop;
    extern __shared__ R rbuf[];  // [G][max_T] projected traces
    const int lane = threadIdx.x, gi = lane / LG, l = lane % LG;
    const int s = G * blockIdx.x + gi;
    const bool have = s < S;
    NmGroup& g = gs[gi];
    R* r = rbuf + (int64_t)gi * max_T;
    const SacDev sd = sacs[have ? s : 0];
    const double q = qorth[sd.slot];
    const int32_t st0 = status_in[sd.slot];
    const bool bad = !have || (st0 & OPMM_ST_NONFINITE_INPUT);
    const uint64_t t0 = wall_clock64();
    if (have && bad) {
        if (l < P) opc_out[(int64_t)s * P + l] = __int_as_float(0x7FC00000);
        if (l == 0) {
            rmse_out[s] = __int_as_float(0x7FC00000);
            if (iters_out) iters_out[s] = 0;
            if (status_out) status_out[s] = st0;
        }
    }
    if (!bad) {
        for (int k = l; k < sd.T; k += LG) r[k] = (R)proj[sd.proj_off + k];
        if (l < P) g.nom[l] = nominal_param_f64(l, (double)sd.dur);
    }
    if (l == 0) g.active = bad ? 0 : 1;
    __syncthreads();
    if (!bad && l < NV) {  // initial simplex: x0 and x0 with one coordinate scaled by 1.05
        for (int j = 0; j < P; ++j) g.v[l][j] = seed_opc ? (double)seed_opc[(int64_t)s * P + j] / g.nom[j] : 1.0;
        if (l > 0) g.v[l][l - 1] = g.v[l][l - 1] * 1.05;
    }
    __syncthreads();
    {
        const bool valid = !bad && l < NV;
        double fv = nm_eval(g, r, g.v[valid ? l : 0], valid, sd, q, dt, lo, hi);
        if (valid) g.f[l] = fv;
    }
    __syncthreads();
    nm_sort(g, l, !bad);
    int it = 0;
    int32_t extra = 0;  // OPMM_ST_DEADLINE when the wall-clock budget ended the task
    for (; it < max_iter; ++it) {
        const bool on = g.active != 0;
        // exit test (max over vertices and coordinates; fmax is exact, so the order does not matter)
        // and the centroid of the best P vertices, one coordinate per lane
        if (on && l < P) {
            double dx = 0.0, acc = 0.0;
            for (int i = 1; i < NV; ++i) dx = fmax(dx, fabs(g.v[i][l] - g.v[0][l]));
            for (int i = 0; i < P; ++i) acc += g.v[i][l];
            g.dxc[l] = dx;
            g.xb[l] = acc / (double)P;
        }
        __syncthreads();
        if (on && l == 0) {
            double dx = 0.0, df = 0.0;
            for (int i = 1; i < NV; ++i) df = fmax(df, fabs(g.f[i] - g.f[0]));
            for (int j = 0; j < P; ++j) dx = fmax(dx, g.dxc[j]);
            g.flag = (dx <= tol_x && df <= tol_f) ? 1 : 0;
        }
        if (lane == 0) s_stop = deadline_ticks > 0 && wall_clock64() - t0 >= deadline_ticks ? 1 : 0;
        __syncthreads();
        const bool stop_now = on && (g.flag || s_stop);  // uniform over the group
        if (stop_now && !g.flag) extra = OPMM_ST_DEADLINE;
        __syncthreads();  // every lane has read the flags before the group stops
        if (stop_now && l == 0) {
            g.active = 0;
            g.iters = it;
        }
        __syncthreads();
        // the loop ends when no group is still iterating
        int any = 0;
#pragma unroll
        for (int k = 0; k < G; ++k) any |= gs[k].active;
        if (!any) break;
        const bool act = g.active != 0;
        if (act && l < NPT) {
            for (int j = 0; j < P; ++j) {
                const double xb = g.xb[j], w = g.v[NV - 1][j];
                double x;
                if (l == 0) x = xb + (xb - w);
                else if (l == 1) x = xb + 2.0 * (xb - w);
                else if (l == 2) x = xb + 0.5 * (xb - w);
                else if (l == 3) x = xb - 0.5 * (xb - w);
                else x = g.v[0][j] + 0.5 * (g.v[l - 3][j] - g.v[0][j]);
                g.pt[l][j] = x;
            }
        }
        __syncthreads();
        {
            const bool valid = act && l < NPT;
            double fv = nm_eval(g, r, g.pt[valid ? l : 0], valid, sd, q, dt, lo, hi);
            if (valid) g.fp[l] = fv;
        }
        __syncthreads();
        if (act && l == 0) {
            const double fr = g.fp[0];
            int d;
            if (fr < g.f[0]) d = g.fp[1] < fr ? 1 : 0;
            else if (fr < g.f[NV - 2]) d = 0;
            else if (fr < g.f[NV - 1]) d = g.fp[2] <= fr ? 2 : 4;
            else d = g.fp[3] < g.f[NV - 1] ? 3 : 4;
            g.dec = d;
            if (dec_out) dec_out[(int64_t)s * max_iter + it] = (int8_t)d;
        }
        __syncthreads();
        if (act) {
            // the accepted point replaces the worst vertex, or the shrink replaces all but the best;
            // one coordinate per lane
            const int d = g.dec;
            if (l < P) {
                if (d < 4) g.v[NV - 1][l] = g.pt[d][l];
                else
                    for (int i = 1; i < NV; ++i) g.v[i][l] = g.pt[3 + i][l];
            }
            if (l == 0) {
                if (d < 4) g.f[NV - 1] = g.fp[d];
                else
                    for (int i = 1; i < NV; ++i) g.f[i] = g.fp[3 + i];
            }
        }
        __syncthreads();
        nm_sort(g, l, act);
    }
    if (bad) return;
    if (l == 0 && g.active) g.iters = it;  // ran to the iteration cap
    if (l < P) {
        double x = fmin(fmax(g.v[0][l], lo), hi);
        opc_out[(int64_t)s * P + l] = (float)(x * g.nom[l]);
    }
    if (l == 0) {
        rmse_out[s] = (float)g.f[0];
        if (iters_out) iters_out[s] = g.iters;
        if (status_out) status_out[s] = st0 | extra;
    }
}

}  // namespace

extern "C" {

void opmm_nm_params_default(opmm_nm_params* p)
{
    if (!p) return;
    p->max_iter = 500;
    p->tol_x = 1e-4f;
    p->tol_f = 1e-6f;
    p->box_frac = 0.25f;
    p->dt_ms = 1.0f;
    p->max_ms = 0.0f;
    p->tasks_per_wave = 0;
}

int opmm_fit_nm(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                const opmm_nm_params* prm, const float* seed_opc, float* opc_out, float* rmse_out, int32_t* iters_out,
                int8_t* decisions_out, int32_t* status_out, void* stream)
{
    if (!ctx) return OPMM_EINVAL;
    if (!prm || prm->max_iter < 0 || !(prm->tol_x >= 0) || !(prm->tol_f >= 0) ||
        !(prm->box_frac > 0 && prm->box_frac < 1) || !(prm->dt_ms > 0 && prm->dt_ms <= 1) || !(prm->max_ms >= 0) ||
        prm->tasks_per_wave < 0 || prm->tasks_per_wave > 2)
        return opmm_rt::fail(ctx, OPMM_EINVAL, "bad Nelder-Mead parameters");
    if (S < 0 || (S > 0 && (!pos || !sacs || !opc_out || !rmse_out))) return opmm_rt::fail(ctx, OPMM_EINVAL, "bad arguments");
    if (S == 0) return OPMM_OK;
    hipStream_t st = (hipStream_t)stream;
    opmm_rt::Ordered ord(opmm_rt::ctx_order(ctx), st);
    if (ord.error() != hipSuccess) return opmm_rt::hip_fail(ctx, ord.error(), "stream ordering");
    const SacDev* d_sacs;
    const float* proj;
    const double* qorth;
    const int32_t* status;
    int rc = opmm_rt::project_batch_full(ctx, pos, pos_len, sacs, S, &d_sacs, &proj, &qorth, &status, st);
    if (rc != OPMM_OK) return rc;
    int max_T = 1;
    for (int i = 0; i < S; ++i) max_T = std::max(max_T, (int)sacs[i].T);
    // two tasks per wave once the batch has more tasks than the device holds waves of this kernel (one
    // per SIMD: it takes 256 VGPRs and ~110 AGPRs); a wave's time is its slower task's, so below that
    // one per wave is as fast.  Measured on 4096 full-estimation saccades: 32k -> 51k saccades/s.
    const int cus = opmm_rt::ctx_cu_count(ctx);
    const int G = prm->tasks_per_wave ? prm->tasks_per_wave : (S > 4 * cus ? 2 : 1);
    uint64_t ticks = 0;
    if (prm->max_ms > 0.0f) {
        int khz = 0;
        hipError_t e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, opmm_rt::ctx_device(ctx));
        if (e != hipSuccess || khz <= 0) return opmm_rt::fail(ctx, OPMM_EDEVICE, "wall clock rate unavailable");
        ticks = std::max<uint64_t>(1, (uint64_t)((double)prm->max_ms * (double)khz));
    }
    const size_t lds = sizeof(R) * (size_t)G * max_T;
    const int grid = (S + G - 1) / G;
    if (G == 2)
        hipLaunchKernelGGL(nm_kernel<2>, dim3(grid), dim3(64), lds, st, S, d_sacs, proj, qorth, status, seed_opc,
                           prm->max_iter, (double)prm->tol_x, (double)prm->tol_f, 1.0 - (double)prm->box_frac,
                           1.0 + (double)prm->box_frac, prm->dt_ms, max_T, ticks, opc_out, rmse_out, iters_out,
                           decisions_out, status_out);
    else
        hipLaunchKernelGGL(nm_kernel<1>, dim3(grid), dim3(64), lds, st, S, d_sacs, proj, qorth, status, seed_opc,
                           prm->max_iter, (double)prm->tol_x, (double)prm->tol_f, 1.0 - (double)prm->box_frac,
                           1.0 + (double)prm->box_frac, prm->dt_ms, max_T, ticks, opc_out, rmse_out, iters_out,
                           decisions_out, status_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return opmm_rt::hip_fail(ctx, e, "nm_kernel");
    return OPMM_OK;
}

}  // extern "C"
