// libopmm: the paper's own estimator -- a parallel Nelder-Mead per saccade
// (Section 3.3, Algorithm 1): one task per saccade, all simplex transforms of
// an iteration evaluated simultaneously, the simplex sorted every iteration,
// both exit tolerances or an iteration cap.
//
// One 64-lane wave per saccade.  The simplex (19 vertices x 18 coordinates,
// FP64, relative to the Table 1 nominal) and the projected trace live in LDS.
// Every iteration lanes 0..21 build and evaluate reflection, expansion, outside
// and inside contraction and the 18 shrink vertices at once; lane 0 takes the
// Lagarias decision (reflection 1, expansion 2, contraction 1/2, shrink 1/2);
// the exit test, the vertex update and the stable re-sort run one coordinate
// or one vertex per lane.  Each evaluation is the same plant
// simulation and RMSE as the box search (points clamped to the search box and
// rounded to FP32, the candidate format).
#include <hip/hip_runtime.h>

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

struct NmSmem {
    R r[OPMM_MAX_T];
    double v[NV][P];
    double f[NV];
    double pt[NPT][P];
    double fp[NPT];
    double xb[P];
    double nom[P];
    double tv[NV][P];  // sort staging
    double tf[NV];
    double dxc[P];     // per-coordinate spread of the simplex
    int flag;
    int dec;
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
__device__ double nm_eval(const NmSmem& sm, const double* x, bool valid, const SacDev& sd, double q, float dt,
                          double lo, double hi)
{
    float p[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double v = valid ? x[j] : 1.0;
        v = fmin(fmax(v, lo), hi);
        p[j] = (float)(v * sm.nom[j]);
    }
    Plant pl;
    plant_setup(p, sd.amp, dt, pl);
    R frac;
    int k0 = pulse_end_sample(pl.pwd, sd.T, frac);
    int kmin = __builtin_amdgcn_readfirstlane(wave_min(valid ? k0 : 0x7FFFFFFF));
    int kmax = __builtin_amdgcn_readfirstlane(wave_max(valid ? k0 : -0x7FFFFFFF));
    SseSinkNm sink{sm.r, 0.0};
    if (valid) run_trajectory<2>(pl, sd.T, (R)dt, k0, frac, kmin, kmax, sink);
    double rm = sqrt((sink.sse + q) / ((double)sd.T * sd.C));
    return (rm >= 0.0 && rm <= 1.7976931348623157e308) ? rm : INFINITY;
}

// Stable sort of the simplex by value, in parallel: vertex i goes to rank
// #{k : f_k < f_i} + #{k < i : f_k == f_i} (the order a stable insertion sort
// gives), each lane moves one row.  Every lane of the wave calls it.
__device__ void nm_sort(NmSmem& sm)
{
    const int lane = threadIdx.x;
    if (lane < NV) {
        const double fi = sm.f[lane];
        int rank = 0;
        for (int k = 0; k < NV; ++k) rank += (sm.f[k] < fi) || (k < lane && sm.f[k] == fi);
        for (int j = 0; j < P; ++j) sm.tv[rank][j] = sm.v[lane][j];
        sm.tf[rank] = fi;
    }
    __syncthreads();
    if (lane < NV) {
        for (int j = 0; j < P; ++j) sm.v[lane][j] = sm.tv[lane][j];
        sm.f[lane] = sm.tf[lane];
    }
    __syncthreads();
}

__global__ __launch_bounds__(64) void nm_kernel(int S, const SacDev* __restrict__ sacs, const float* __restrict__ proj,
                                                const double* __restrict__ qorth, const int32_t* __restrict__ status_in,
                                                const float* __restrict__ seed_opc, int max_iter, double tol_x,
                                                double tol_f, double lo, double hi, float dt, float* opc_out,
                                                float* rmse_out, int32_t* iters_out, int8_t* dec_out,
                                                int32_t* status_out)
{
    __shared__ NmSmem sm;
    const int s = blockIdx.x, lane = threadIdx.x;
    const SacDev sd = sacs[s];
    const double q = qorth[sd.slot];
    const int32_t st0 = status_in[sd.slot];
    if (st0 & OPMM_ST_NONFINITE_INPUT) {
        if (lane < P) opc_out[(int64_t)s * P + lane] = __int_as_float(0x7FC00000);
        if (lane == 0) {
            rmse_out[s] = __int_as_float(0x7FC00000);
            if (iters_out) iters_out[s] = 0;
            if (status_out) status_out[s] = st0;
        }
        return;
    }
    for (int k = lane; k < sd.T; k += 64) sm.r[k] = (R)proj[sd.proj_off + k];
    if (lane < P) sm.nom[lane] = nominal_param_f64(lane, (double)sd.dur);
    __syncthreads();
    if (lane < NV) {  // initial simplex: x0 and x0 with one coordinate scaled by 1.05
        for (int j = 0; j < P; ++j)
            sm.v[lane][j] = seed_opc ? (double)seed_opc[(int64_t)s * P + j] / sm.nom[j] : 1.0;
        if (lane > 0) sm.v[lane][lane - 1] = sm.v[lane][lane - 1] * 1.05;
    }
    __syncthreads();
    {
        double fv = nm_eval(sm, sm.v[lane < NV ? lane : 0], lane < NV, sd, q, dt, lo, hi);
        if (lane < NV) sm.f[lane] = fv;
    }
    __syncthreads();
    nm_sort(sm);
    int it = 0;
    for (; it < max_iter; ++it) {
        // exit test (max over vertices and coordinates; fmax is exact, so the order does not matter)
        // and the centroid of the best P vertices, one coordinate per lane
        if (lane < P) {
            double dx = 0.0, acc = 0.0;
            for (int i = 1; i < NV; ++i) dx = fmax(dx, fabs(sm.v[i][lane] - sm.v[0][lane]));
            for (int i = 0; i < P; ++i) acc += sm.v[i][lane];
            sm.dxc[lane] = dx;
            sm.xb[lane] = acc / (double)P;
        }
        __syncthreads();
        if (lane == 0) {
            double dx = 0.0, df = 0.0;
            for (int i = 1; i < NV; ++i) df = fmax(df, fabs(sm.f[i] - sm.f[0]));
            for (int j = 0; j < P; ++j) dx = fmax(dx, sm.dxc[j]);
            sm.flag = (dx <= tol_x && df <= tol_f) ? 1 : 0;
        }
        __syncthreads();
        if (sm.flag) break;
        if (lane < NPT) {
            for (int j = 0; j < P; ++j) {
                const double xb = sm.xb[j], w = sm.v[NV - 1][j];
                double x;
                if (lane == 0) x = xb + (xb - w);
                else if (lane == 1) x = xb + 2.0 * (xb - w);
                else if (lane == 2) x = xb + 0.5 * (xb - w);
                else if (lane == 3) x = xb - 0.5 * (xb - w);
                else x = sm.v[0][j] + 0.5 * (sm.v[lane - 3][j] - sm.v[0][j]);
                sm.pt[lane][j] = x;
            }
        }
        __syncthreads();
        {
            double fv = nm_eval(sm, sm.pt[lane < NPT ? lane : 0], lane < NPT, sd, q, dt, lo, hi);
            if (lane < NPT) sm.fp[lane] = fv;
        }
        __syncthreads();
        if (lane == 0) {
            const double fr = sm.fp[0];
            int d;
            if (fr < sm.f[0]) d = sm.fp[1] < fr ? 1 : 0;
            else if (fr < sm.f[NV - 2]) d = 0;
            else if (fr < sm.f[NV - 1]) d = sm.fp[2] <= fr ? 2 : 4;
            else d = sm.fp[3] < sm.f[NV - 1] ? 3 : 4;
            sm.dec = d;
            if (dec_out) dec_out[(int64_t)s * max_iter + it] = (int8_t)d;
        }
        __syncthreads();
        {
            // the accepted point replaces the worst vertex, or the shrink replaces all but the best;
            // one coordinate per lane
            const int d = sm.dec;
            if (lane < P) {
                if (d < 4) sm.v[NV - 1][lane] = sm.pt[d][lane];
                else
                    for (int i = 1; i < NV; ++i) sm.v[i][lane] = sm.pt[3 + i][lane];
            }
            if (lane == 0) {
                if (d < 4) sm.f[NV - 1] = sm.fp[d];
                else
                    for (int i = 1; i < NV; ++i) sm.f[i] = sm.fp[3 + i];
            }
        }
        __syncthreads();
        nm_sort(sm);
    }
    if (lane < P) {
        double x = fmin(fmax(sm.v[0][lane], lo), hi);
        opc_out[(int64_t)s * P + lane] = (float)(x * sm.nom[lane]);
    }
    if (lane == 0) {
        rmse_out[s] = (float)sm.f[0];
        if (iters_out) iters_out[s] = it;
        if (status_out) status_out[s] = st0;
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
}

int opmm_fit_nm(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                const opmm_nm_params* prm, const float* seed_opc, float* opc_out, float* rmse_out, int32_t* iters_out,
                int8_t* decisions_out, int32_t* status_out, void* stream)
{
    if (!ctx) return OPMM_EINVAL;
    if (!prm || prm->max_iter < 0 || !(prm->tol_x >= 0) || !(prm->tol_f >= 0) ||
        !(prm->box_frac > 0 && prm->box_frac < 1) || !(prm->dt_ms > 0 && prm->dt_ms <= 1))
        return opmm_rt::fail(ctx, OPMM_EINVAL, "bad Nelder-Mead parameters");
    if (S < 0 || (S > 0 && (!pos || !sacs || !opc_out || !rmse_out))) return opmm_rt::fail(ctx, OPMM_EINVAL, "bad arguments");
    if (S == 0) return OPMM_OK;
    hipStream_t st = (hipStream_t)stream;
    const SacDev* d_sacs;
    const float* proj;
    const double* qorth;
    const int32_t* status;
    int rc = opmm_rt::project_batch_full(ctx, pos, pos_len, sacs, S, &d_sacs, &proj, &qorth, &status, st);
    if (rc != OPMM_OK) return rc;
    hipLaunchKernelGGL(nm_kernel, dim3(S), dim3(64), 0, st, S, d_sacs, proj, qorth, status, seed_opc, prm->max_iter,
                       (double)prm->tol_x, (double)prm->tol_f, 1.0 - (double)prm->box_frac, 1.0 + (double)prm->box_frac,
                       prm->dt_ms, opc_out, rmse_out, iters_out, decisions_out, status_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return opmm_rt::hip_fail(ctx, e, "nm_kernel");
    return OPMM_OK;
}

}  // extern "C"
