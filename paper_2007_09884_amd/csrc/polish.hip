// libopmm: gradient-based estimation -- the alternative to the simplex search
// that the paper leaves to future work (Section 5) -- as a polish after the
// box search, with exact forward sensitivities of the plant.
//
// Sensitivities.  The plant is linear and time-invariant on each piece of the
// pulse-step control (Section 2.1), so theta_k is a smooth function of the OPC
// p (PW included: it moves the switching instant inside its sample).  The
// derivative d theta_k / d p_j is computed in forward mode: the plant's scalar
// physics (the same template as the search path), the one-sample transition
// of each piece, the exact split of the pulse-end sample and the recurrence
// all run on dual numbers (value, derivative) seeded with the unit direction
// of parameter j.  One lane per parameter, one wave per saccade.  The
// sensitivity entry point's discretisation (Taylor degree 12 on dt/4 and two
// squarings; degree 20 for the split) truncates below 1e-11 relative even for
// the fastest mechanical mode in a +/-25% box (~2.6 per ms), so these are the
// sensitivities of the exact trajectory to that accuracy.
//
// Polish.  Levenberg-Marquardt on the fit cost with Marquardt's diagonal
// scaling, in coordinates relative to the Table 1 nominal.  Every iteration
// forms J^T W J and J^T W e from a sensitivity pass on the search path's
// discretisation (it only shapes the step), then 8 lanes solve the damped
// system for 8 damping values at once (lambda_c * 10^(m-4), m = 0..7;
// Cholesky per lane) and evaluate their trial points, and a ninth lane the
// cost at the current point, all on the exact discretisation; the best trial
// is taken if it lowers the cost (lambda_c becomes a tenth of its lambda),
// otherwise lambda_c grows by 1e8 and the point stays.
// A wave polishes one, two or three saccades, one lane group each (64, 32 or 21 lanes: a saccade
// alone leaves 46 lanes idle in the Jacobian pass and 55 in the trial pass, but its wave finishes
// sooner).  Each group's arithmetic is exactly that of a wave of its own.  The launch picks the
// layout with the least time from the waves per SIMD and the measured relative wave times: large
// batches share waves; batches that fit one wave per SIMD, and batches holding a trace longer than
// 512 samples (three staged traces would not leave room for four waves per CU), do not.
// Objectives: the RMSE of Section 3.4 (Gauss-Newton on squared residuals) or
// the mean absolute difference the paper reports as OptErr (Fig. 4), by
// iteratively reweighted least squares (weights 1/max(|e|, 1e-3 deg)).
// Parameters at a bound whose gradient points outward are held; trial points
// are clamped to the search box and rounded to FP32, the candidate format.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/opmm.h"
#include "plant.hpp"
#include "runtime.hpp"

namespace opmm {

// Forward-mode dual number: value and derivative along one direction.  Value
// parts follow exactly the double operations of the plain path.
struct Dual {
    double v, d;
    Dual() = default;
    __device__ constexpr Dual(double x) : v(x), d(0.0) {}
    __device__ constexpr Dual(double x, double dx) : v(x), d(dx) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, __fma_rn(a.v, b.d, a.d * b.v)); }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
__device__ __forceinline__ Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
__device__ __forceinline__ Dual fmr(Dual a, Dual b, Dual c)
{
    return Dual(__fma_rn(a.v, b.v, c.v), __fma_rn(a.v, b.d, __fma_rn(a.d, b.v, c.d)));
}
__device__ __forceinline__ Dual rcp64(Dual a)
{
    const double r = rcp64(a.v);
    return Dual(r, -a.d * r * r);
}
__device__ __forceinline__ double val(double a) { return a; }
__device__ __forceinline__ double val(Dual a) { return a.v; }

}  // namespace opmm

using namespace opmm;
using opmm_rt::SacDev;

namespace {

constexpr int NLAM = 8;             // damping values tried per iteration
constexpr int PTRI = P * (P + 1) / 2;
constexpr double IRLS_EPS = 1e-3;   // deg: floor of |e| in the L1 weights
constexpr int NCH = 32;             // samples of Jacobian rows staged in LDS per normal-equation pass
// Lane groups: a wave polishes pg saccades, group_lanes(pg) lanes each (P sensitivity directions
// in the Jacobian pass, NLAM + 1 cost lanes in the trial pass).
constexpr int group_lanes(int pg) { return pg == 1 ? 64 : pg == 2 ? 32 : 21; }
static_assert(group_lanes(3) >= P && group_lanes(3) >= NLAM + 1 && 3 * group_lanes(3) <= 64, "lane groups");
// traces up to this length may share a wave (three staged traces leave room for four waves per CU)
constexpr int GROUPED_MAX_T = 512;
// Discretisations of the plant: Taylor degree M and squarings SQ of the
// one-sample transition (on dt / 2^SQ), Taylor degree EXM of the split
// sample's exponentials.  Exact: truncation below 1e-11 relative for the
// fastest mechanical mode of a +/-25% box (~2.6 per ms).  Fast: the search
// path's (~1e-8 deg on trajectories), enough for a Gauss-Newton model.
struct DiscExact { static constexpr int M = 12, SQ = 2, EXM = 20; };
struct DiscFast { static constexpr int M = 6, SQ = 2, EXM = 11; };
// damping factors of the 8 trial lanes, relative to the current lambda
__constant__ double LAM_FAC[NLAM] = {1e-4, 1e-3, 1e-2, 1e-1, 1.0, 1e1, 1e2, 1e3};

// D-form transition of one piece: mechanical block, coupling to (F_ag, F_ant),
// active-state factors minus one.
template <class S>
struct Piece {
    S m[4][4], x[4][2], e[2];
};

// rows of Mc * V for the mechanical block Mc (theta' = omega is row 0)
template <class S>
__device__ __forceinline__ void mech_rows(const PlantScalars<S>& c, const S v[4], S o[4])
{
    o[0] = v[1];
    o[1] = fmr(c.a13, v[3], fmr(c.a12, v[2], fmr(c.a11, v[1], c.a10 * v[0])));
    o[2] = fmr(c.a22, v[2], c.a20 * v[0]);
    o[3] = fmr(c.a33, v[3], c.a30 * v[0]);
}

// D = exp(dt A) - I of the piece with active-state rates (qa, qn): Horner
// evaluation of the degree-M Taylor polynomial on h = dt / 2^SQ in block form
// A = [[Mc, G], [0, diag(q)]], then SQ squarings D_2h = D_h^2 + 2 D_h.
template <int M, int SQ, class S>
__device__ void lti_dform(const PlantScalars<S>& c, S qa, S qn, double dt, Piece<S>& o)
{
    const double h = dt / (double)(1 << SQ);
    const S q[2] = {qa, qn};
    S qm[4][4], qx[4][2], qd[2];
    for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) qm[i][j] = S(i == j ? 1.0 : 0.0);
        qx[i][0] = S(0.0); qx[i][1] = S(0.0);
    }
    qd[0] = S(1.0); qd[1] = S(1.0);
    for (int k = M; k >= 1; --k) {
        // Q <- I + (h/k) A Q  (k >= 2);  D = h A Q  (k == 1)
        const double s = h / (double)k;
        S am[4][4], ax[4][2], ad[2];
        for (int col = 0; col < 4; ++col) {
            S v[4] = {qm[0][col], qm[1][col], qm[2][col], qm[3][col]}, r[4];
            mech_rows(c, v, r);
            for (int i = 0; i < 4; ++i) am[i][col] = r[i];
        }
        for (int col = 0; col < 2; ++col) {
            S v[4] = {qx[0][col], qx[1][col], qx[2][col], qx[3][col]}, r[4];
            mech_rows(c, v, r);
            for (int i = 0; i < 4; ++i) ax[i][col] = r[i];
        }
        ax[2][0] = fmr(c.g2, qd[0], ax[2][0]);
        ax[3][1] = fmr(c.g3, qd[1], ax[3][1]);
        ad[0] = q[0] * qd[0];
        ad[1] = q[1] * qd[1];
        const double one = k >= 2 ? 1.0 : 0.0;
        for (int i = 0; i < 4; ++i) {
            for (int j = 0; j < 4; ++j) qm[i][j] = fmr(S(s), am[i][j], S(i == j ? one : 0.0));
            qx[i][0] = S(s) * ax[i][0];
            qx[i][1] = S(s) * ax[i][1];
        }
        qd[0] = fmr(S(s), ad[0], S(one));
        qd[1] = fmr(S(s), ad[1], S(one));
    }
    // squarings in D-form
    for (int q = 0; q < SQ; ++q) {
        S nm[4][4], nx[4][2];
        for (int i = 0; i < 4; ++i) {
            for (int j = 0; j < 4; ++j) {
                S a = qm[i][j] + qm[i][j];
                for (int k = 0; k < 4; ++k) a = fmr(qm[i][k], qm[k][j], a);
                nm[i][j] = a;
            }
            for (int j = 0; j < 2; ++j) {
                S b = qx[i][j] * (qd[j] + S(2.0));
                for (int k = 0; k < 4; ++k) b = fmr(qm[i][k], qx[k][j], b);
                nx[i][j] = b;
            }
        }
        for (int i = 0; i < 4; ++i) {
            for (int j = 0; j < 4; ++j) qm[i][j] = nm[i][j];
            qx[i][0] = nx[i][0];
            qx[i][1] = nx[i][1];
        }
        qd[0] = qd[0] * (qd[0] + S(2.0));
        qd[1] = qd[1] * (qd[1] + S(2.0));
    }
    for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) o.m[i][j] = qm[i][j];
        o.x[i][0] = qx[i][0];
        o.x[i][1] = qx[i][1];
    }
    o.e[0] = qd[0];
    o.e[1] = qd[1];
}

template <class S>
__device__ __forceinline__ void piece_step(const Piece<S>& pc, S d[6])
{
    S n[4];
    for (int i = 0; i < 4; ++i) {
        S a = d[i];
        for (int j = 0; j < 4; ++j) a = fmr(pc.m[i][j], d[j], a);
        a = fmr(pc.x[i][0], d[4], a);
        n[i] = fmr(pc.x[i][1], d[5], a);
    }
    d[4] = fmr(pc.e[0], d[4], d[4]);
    d[5] = fmr(pc.e[1], d[5], d[5]);
    for (int i = 0; i < 4; ++i) d[i] = n[i];
}

// v <- exp(t A) v by the Taylor polynomial of degree EXM (|t| <= dt)
template <int EXM, class S>
__device__ void expmv_t(const PlantScalars<S>& c, S qa, S qn, S t, S v[6])
{
    S w[6];
    for (int i = 0; i < 6; ++i) w[i] = v[i];
    for (int k = EXM; k >= 1; --k) {
        const S s = t * (1.0 / (double)k);
        S mv[4], aw[6];
        S w4[4] = {w[0], w[1], w[2], w[3]};
        mech_rows(c, w4, mv);
        aw[0] = mv[0];
        aw[1] = mv[1];
        aw[2] = fmr(c.g2, w[4], mv[2]);
        aw[3] = fmr(c.g3, w[5], mv[3]);
        aw[4] = qa * w[4];
        aw[5] = qn * w[5];
        for (int i = 0; i < 6; ++i) w[i] = fmr(s, aw[i], v[i]);
    }
    for (int i = 0; i < 6; ++i) v[i] = w[i];
}

// theta_k, k = 0..T-1, of OPC p (deg), handed to sink(k, theta_k), with the
// discretisation Disc.  Control flow depends on value parts only, so every
// lane of a Dual pass at one point takes the same path.
template <class Disc, class S, class Sink>
__device__ void simulate_s(const S p[P], double amp, double dt, int T, Sink& sink)
{
    PlantScalars<S> c;
    plant_scalars(p, S(amp), c);
    const S pwd = p[17] * rcp64(dt);
    const double fl = floor(val(pwd));
    int k0;
    S frac(0.0);
    if (!(val(pwd) > 0.0)) k0 = -1;
    else if (fl >= (double)T) k0 = T;
    else { k0 = (int)fl; frac = pwd - S(fl); }
    S d[6];
    for (int i = 0; i < 6; ++i) d[i] = c.d0[i];
    S theq = c.th1;
    // one piece's transition at a time (the post piece is formed when the pulse ends), which
    // keeps the dual pass within the register file
    Piece<S> pc;
    int k = 0;
    if (k0 < 0) {
        for (int i = 0; i < 6; ++i) d[i] = d[i] + c.sh[i];
        theq = S(amp);
    } else {
        lti_dform<Disc::M, Disc::SQ>(c, c.q1a, c.q1n, dt, pc);
        for (; k < k0 && k < T; ++k) {
            sink(k, d[0] + theq);
            piece_step(pc, d);
        }
        if (k0 >= T) return;
        sink(k, d[0] + theq);
        expmv_t<Disc::EXM>(c, c.q1a, c.q1n, frac * dt, d);
        for (int i = 0; i < 6; ++i) d[i] = d[i] + c.sh[i];
        expmv_t<Disc::EXM>(c, c.q2a, c.q2n, (S(1.0) - frac) * dt, d);
        theq = S(amp);
        ++k;
    }
    lti_dform<Disc::M, Disc::SQ>(c, c.q2a, c.q2n, dt, pc);
    for (; k < T; ++k) {
        sink(k, d[0] + theq);
        piece_step(pc, d);
    }
}

// ---- sinks ----------------------------------------------------------------

struct JacSink {  // theta and d theta / d p_lane
    double* theta;
    double* jac;  // [T][P] row-major
    int lane;
    __device__ void operator()(int k, Dual th)
    {
        if (lane == 0) theta[k] = th.v;
        if (lane < P) jac[(int64_t)k * P + lane] = th.d;
    }
};

struct Residual {
    const float* X;
    const float* Y;
    double cphi, sphi;
    int C;
    __device__ __forceinline__ void operator()(int k, double th, double& ex, double& ey) const
    {
        ex = th * cphi - (double)X[k];
        ey = C == 2 ? th * sphi - (double)Y[k] : 0.0;
    }
};

struct CostSink {  // objective value only (trial points, reports)
    Residual res;
    int objective;
    double sq, ab;
    __device__ void operator()(int k, double th)
    {
        double ex, ey;
        res(k, th, ex, ey);
        sq = __fma_rn(ex, ex, sq);
        ab += fabs(ex);
        if (res.C == 2) {
            sq = __fma_rn(ey, ey, sq);
            ab += fabs(ey);
        }
    }
    __device__ double f() const { return objective == OPMM_OBJ_MAE ? ab : sq; }
};

// Orders LDS accesses among the lanes of the wave (a block is one wave).  Lane groups flush at
// different samples, so no block barrier may be used there.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Normal equations of the linearised problem.  Lane r of the saccade's group carries column r of
// J (the dual part) and accumulates g_r; the rows of J are staged in LDS NCH samples at a time,
// and each lane of the group then accumulates up to NENT entries (i >= j) of the lower triangle
// of J^T W J, h_ij += (w_k J_ki) J_kj in sample order.  Every lane of the group calls it (the
// group's control flow is uniform).
template <int GL>
struct NormalSink {
    static constexpr int NENT = (PTRI + GL - 1) / GL;  // lower-triangle entries accumulated per lane
    Residual res;
    int objective;
    double* jst;  // LDS [NCH][P]: staged rows of J
    double* ast;  // LDS [NCH]: per-sample weight of the normal matrix
    int r;        // lane within the group
    int nk;       // samples staged
    double g;
    int eij[NENT];  // this lane's entries, (row << 8) | column; -1: none
    double h[NENT];
    __device__ void init(int nf)
    {
        nk = 0;
        g = 0.0;
#pragma unroll
        for (int q = 0; q < NENT; ++q) {
            const int e = r + GL * q;
            int i = 0;
            while ((i + 1) * (i + 2) / 2 <= e) ++i;
            const bool use = e < PTRI && i < nf;
            eij[q] = use ? (i << 8) | (e - i * (i + 1) / 2) : -1;
            h[q] = 0.0;
        }
    }
    __device__ void operator()(int k, Dual th)
    {
        double ex, ey;
        res(k, th.v, ex, ey);
        double wx = 1.0, wy = 1.0;
        if (objective == OPMM_OBJ_MAE) {
            wx = 1.0 / fmax(fabs(ex), IRLS_EPS);
            wy = 1.0 / fmax(fabs(ey), IRLS_EPS);
        }
        const double cp = res.cphi, sp = res.sphi;
        double a = wx * cp * cp, b = wx * cp * ex;
        if (res.C == 2) {
            a = __fma_rn(wy * sp, sp, a);
            b = __fma_rn(wy * sp, ey, b);
        }
        g = __fma_rn(th.d, b, g);
        if (r < P) jst[nk * P + r] = th.d;
        if (r == 0) ast[nk] = a;
        if (++nk == NCH) flush();
    }
    __device__ void flush()
    {
        wave_sync();
        for (int kk = 0; kk < nk; ++kk) {
            const double ak = ast[kk];
#pragma unroll
            for (int q = 0; q < NENT; ++q)
                if (eij[q] >= 0)
                    h[q] = __fma_rn(ak * jst[kk * P + (eij[q] >> 8)], jst[kk * P + (eij[q] & 255)], h[q]);
        }
        wave_sync();
        nk = 0;
    }
};

// ---- sensitivity entry point ------------------------------------------------

__global__ __launch_bounds__(64) void sensitivity_kernel(int S, const SacDev* __restrict__ sacs,
                                                         const int64_t* __restrict__ out_off,
                                                         const float* __restrict__ opc, double dt,
                                                         double* __restrict__ theta, double* __restrict__ jac)
{
    const int s = blockIdx.x, lane = threadIdx.x;
    const SacDev sd = sacs[s];
    Dual p[P];
#pragma unroll
    for (int j = 0; j < P; ++j) p[j] = Dual((double)opc[(int64_t)s * P + j], j == lane ? 1.0 : 0.0);
    JacSink sink{theta + out_off[s], jac + out_off[s] * P, lane};
    simulate_s<DiscExact>(p, (double)sd.amp, dt, sd.T, sink);
}

// ---- polish -------------------------------------------------------------------

// State of one saccade's polish (one lane group).
struct PolishSlot {
    double H[P][P];
    double g[P];
    double xt[NLAM][P];
    double ft[NLAM];
    double x[P], nom[P], lo[P], hi[P];
    double jst[NCH][P];
    double ast[NCH];
    int opc_of[P];   // free parameter -> its (first) OPC index
    int tied[P];     // free parameter -> second OPC index it moves, or -1
    int nf;
    double fcur, lam;
    int ok[NLAM];
    int done;        // no further iterations (converged, stopped, or no saccade in the group)
    int it;          // iterations taken
};

// OPC of relative point x, rounded to FP32 (the candidate format)
__device__ __forceinline__ double opc_value(const PolishSlot& sl, const double* x, int i)
{
    return (double)(float)(x[i] * sl.nom[i]);
}

// Cholesky solve of (H + lam diag H) delta = -g with the factor in registers
// (fully unrolled, 18 unknowns).  Unknowns flagged in `held` (held parameters
// and those past the free count) take an identity row, so their delta is 0.
// The diagonal of the packed factor stores 1/L_jj.  Returns false if the
// damped matrix is not positive definite.
__device__ __forceinline__ bool damped_solve(const PolishSlot& sl, double lam, uint32_t held, double delta[P])
{
    double L[PTRI];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const bool uj = !((held >> j) & 1u);
        double d = uj ? sl.H[j][j] * (1.0 + lam) : 1.0;
#pragma unroll
        for (int k = 0; k < j; ++k) d = __fma_rn(-L[j * (j + 1) / 2 + k], L[j * (j + 1) / 2 + k], d);
        if (!(d > 0.0)) return false;
        const double rj = 1.0 / sqrt(d);
        L[j * (j + 1) / 2 + j] = rj;
#pragma unroll
        for (int i = j + 1; i < P; ++i) {
            const bool ui = !((held >> i) & 1u);
            double a = (ui && uj) ? sl.H[i][j] : 0.0;
#pragma unroll
            for (int k = 0; k < j; ++k) a = __fma_rn(-L[i * (i + 1) / 2 + k], L[j * (j + 1) / 2 + k], a);
            L[i * (i + 1) / 2 + j] = a * rj;
        }
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {  // L y = -g
        double a = ((held >> i) & 1u) ? 0.0 : -sl.g[i];
#pragma unroll
        for (int k = 0; k < i; ++k) a = __fma_rn(-L[i * (i + 1) / 2 + k], delta[k], a);
        delta[i] = a * L[i * (i + 1) / 2 + i];
    }
#pragma unroll
    for (int i = P - 1; i >= 0; --i) {  // L^T delta = y
        double a = delta[i];
#pragma unroll
        for (int k = i + 1; k < P; ++k) a = __fma_rn(-L[k * (k + 1) / 2 + i], delta[k], a);
        delta[i] = a * L[i * (i + 1) / 2 + i];
    }
    return true;
}

// PG saccades per wave: lane group g = lane / GL polishes saccade order[blockIdx.x * PG + g]
// (order: the batch sorted by T, so a wave's saccades run loops of similar length; NULL: batch
// order).  A group's arithmetic is that of a wave of its own, so results do not depend on the
// grouping.  Traces are staged in dynamic LDS, [PG][2][max_T] floats; max_T bounds every T.
template <int PG>
__global__ __launch_bounds__(64) void polish_kernel(int S, const SacDev* __restrict__ sacs,
                                                    const int* __restrict__ order, const float* __restrict__ pos,
                                                    const int32_t* __restrict__ status_in, int max_T, int model,
                                                    int max_iter, int objective, double tol_f, double lam0,
                                                    double box_frac, double dt, float* __restrict__ opc,
                                                    float* __restrict__ rmse_out, float* __restrict__ mae_out,
                                                    int32_t* __restrict__ iters_out, int8_t* __restrict__ dec_out)
{
    __shared__ PolishSlot slots[PG];
    extern __shared__ float traces[];
    const int lane = threadIdx.x;
    constexpr int GL = group_lanes(PG);
    const bool member = lane < PG * GL;
    const int g = member ? lane / GL : 0;
    const int r = lane - g * GL;  // lanes past the groups have r >= GL and no role
    const int idx = blockIdx.x * PG + g;
    const bool has = member && idx < S;
    const int s = has ? (order ? order[idx] : idx) : 0;
    PolishSlot& sl = slots[g];
    float* X = traces + (size_t)g * 2 * max_T;
    float* Y = X + max_T;
    const SacDev sd = has ? sacs[s] : SacDev{};
    const int T = sd.T;
    bool live = has;
    if (has && ((status_in[sd.slot] & OPMM_ST_NONFINITE_INPUT) || T > max_T)) {
        if (r < P) opc[(int64_t)s * P + r] = __int_as_float(0x7FC00000);
        if (r == 0) {
            rmse_out[s] = __int_as_float(0x7FC00000);
            if (mae_out) mae_out[s] = __int_as_float(0x7FC00000);
            if (iters_out) iters_out[s] = 0;
        }
        live = false;
    }
    if (live) {
        for (int k = r; k < T; k += GL) {
            X[k] = pos[sd.pos_off + (int64_t)k * sd.C];
            Y[k] = sd.C == 2 ? pos[sd.pos_off + (int64_t)k * sd.C + 1] : 0.0f;
        }
        if (r < P) {
            const double nm = nominal_param_f64(r, (double)sd.dur);
            const double v = (double)opc[(int64_t)s * P + r];
            sl.nom[r] = nm;
            sl.x[r] = v / nm;
            const bool fixed = model == 9 && fixed_in_model9(r);
            sl.lo[r] = fixed ? sl.x[r] : 1.0 - box_frac;
            sl.hi[r] = fixed ? sl.x[r] : 1.0 + box_frac;
        }
    }
    if (member && r == 0) {
        int n = 0;
        for (int i = 0; i < P && live; ++i) {
            if (model == 9 && (fixed_in_model9(i) || i == 1 || i == 3)) continue;
            sl.opc_of[n] = i;
            sl.tied[n] = (model == 9 && (i == 0 || i == 2)) ? i + 1 : -1;
            ++n;
        }
        sl.nf = n;
        sl.lam = lam0;
        sl.done = live ? 0 : 1;
        sl.it = live ? max_iter : 0;
    }
    __syncthreads();
    if (live && r < P) {
        // 9-parameter model: the antagonist's K_SE and K_LT follow the agonist's
        const int src = (model == 9 && (r == 1 || r == 3)) ? r - 1 : r;
        const double v = opc_value(sl, sl.x, src) / sl.nom[r];
        sl.x[r] = fmin(fmax(model == 9 ? v : sl.x[r], sl.lo[r]), sl.hi[r]);
    }
    __syncthreads();
    const int nf = sl.nf;
    const Residual res{X, Y, sd.cphi, sd.sphi, sd.C};
    for (int it = 0; it < max_iter; ++it) {
        bool all_done = true;
        for (int q = 0; q < PG; ++q) all_done = all_done && slots[q].done;
        if (all_done) break;
        const bool run = live && !sl.done;
        // A: sensitivities and normal equations at x (lane r: free parameter r), on the fast
        // discretisation: it only shapes the step; costs below are exact
        if (run) {
            Dual p[P];
            const int i0 = r < nf ? sl.opc_of[r] : -1;
            const int i1 = r < nf ? sl.tied[r] : -1;
            for (int i = 0; i < P; ++i)
                p[i] = Dual(opc_value(sl, sl.x, i), (i == i0 || i == i1) ? sl.nom[i] : 0.0);
            NormalSink<GL> ns{res, objective, &sl.jst[0][0], sl.ast, r};
            ns.init(nf);
            simulate_s<DiscFast>(p, (double)sd.amp, dt, T, ns);
            ns.flush();
#pragma unroll
            for (int q = 0; q < NormalSink<GL>::NENT; ++q)
                if (ns.eij[q] >= 0) sl.H[ns.eij[q] >> 8][ns.eij[q] & 255] = ns.h[q];
            if (r < nf) sl.g[r] = ns.g;
        }
        __syncthreads();
        // B: damped solves, one damping value per lane
        if (run && r < NLAM) {
            const double lam = sl.lam * LAM_FAC[r];
            uint32_t held = 0;
            for (int j = 0; j < P; ++j) {
                bool h = true;
                if (j < nf) {
                    const int i = sl.opc_of[j];
                    h = !(sl.H[j][j] > 0.0) || (sl.x[i] <= sl.lo[i] && sl.g[j] > 0.0) ||
                        (sl.x[i] >= sl.hi[i] && sl.g[j] < 0.0);
                }
                held |= (uint32_t)h << j;
            }
            double delta[P];
            const bool ok = damped_solve(sl, lam, held, delta);
            for (int i = 0; i < P; ++i) sl.xt[r][i] = sl.x[i];
            if (ok) {
                for (int j = 0; j < nf; ++j) {
                    const int i = sl.opc_of[j];
                    const double v = fmin(fmax(sl.x[i] + delta[j], sl.lo[i]), sl.hi[i]);
                    sl.xt[r][i] = v;
                    if (sl.tied[j] >= 0) sl.xt[r][sl.tied[j]] = v;
                }
            }
            sl.ok[r] = ok;
            sl.ft[r] = INFINITY;
        }
        __syncthreads();
        // C: trial costs, and the cost at the current point (lane NLAM)
        if (run && ((r < NLAM && sl.ok[r]) || r == NLAM)) {
            const double* xp = r < NLAM ? sl.xt[r] : sl.x;
            double p[P];
            for (int i = 0; i < P; ++i) p[i] = opc_value(sl, xp, i);
            CostSink cs{res, objective, 0.0, 0.0};
            simulate_s<DiscExact>(p, (double)sd.amp, dt, T, cs);
            const double f = cs.f();
            if (r < NLAM) sl.ft[r] = (f >= 0.0 && f <= 1.7976931348623157e308) ? f : INFINITY;
            else sl.fcur = f;
        }
        __syncthreads();
        // D: decision
        if (run && r == 0) {
            int best = 0;
            for (int m = 1; m < NLAM; ++m)
                if (sl.ft[m] < sl.ft[best]) best = m;
            int dec;
            if (sl.ft[best] < sl.fcur) {
                dec = best;
                const double gain = sl.fcur - sl.ft[best];
                for (int i = 0; i < P; ++i) sl.x[i] = sl.xt[best][i];
                sl.lam = sl.lam * LAM_FAC[best] * 0.1;
                sl.done = gain <= tol_f * sl.ft[best];
            } else {
                dec = -1;
                sl.lam *= 1e8;
                sl.done = !(sl.lam <= 1e30);
            }
            if (sl.done) sl.it = it + 1;
            if (dec_out) dec_out[(int64_t)s * max_iter + it] = (int8_t)dec;
        }
        __syncthreads();
    }
    if (live && r < P) opc[(int64_t)s * P + r] = (float)opc_value(sl, sl.x, r);
    if (live && r == 0) {
        double p[P];
        for (int i = 0; i < P; ++i) p[i] = opc_value(sl, sl.x, i);
        CostSink cs{res, objective, 0.0, 0.0};
        simulate_s<DiscExact>(p, (double)sd.amp, dt, T, cs);
        const double n = (double)T * sd.C;
        rmse_out[s] = (float)sqrt(cs.sq / n);
        if (mae_out) mae_out[s] = (float)(cs.ab / n);
        if (iters_out) iters_out[s] = sl.it;
    }
}

// Time of one wave polishing pg saccades, relative to a wave with one (measured with one wave per
// SIMD: the groups' loops run to the longest member, and each lane accumulates more entries of
// the normal matrix).
constexpr double WAVE_TIME[4] = {0.0, 1.0, 1.30, 1.51};

// Saccades per wave for n saccades (T <= max_T) on `simds` SIMDs: one wave per SIMD is resident at
// a time, so a batch takes ceil(waves / simds) wave times.
int polish_group(int n, int max_T, int simds)
{
    if (max_T > GROUPED_MAX_T) return 1;
    int best = 1;
    double best_t = 0.0;
    for (int pg = 1; pg <= 3; ++pg) {
        const int64_t waves = ((int64_t)n + pg - 1) / pg;
        const double t = (double)((waves + simds - 1) / simds) * WAVE_TIME[pg];
        if (pg == 1 || t < best_t) {
            best = pg;
            best_t = t;
        }
    }
    return best;
}

template <int PG>
void launch_group(const SacDev* sacs, const int* order, int n, int max_T, const float* pos, const int32_t* status,
                  int model, const opmm_polish_params& prm, float* opc, float* rmse, float* mae, int32_t* iters,
                  int8_t* dec, hipStream_t st)
{
    hipLaunchKernelGGL(polish_kernel<PG>, dim3((n + PG - 1) / PG), dim3(64), sizeof(float) * 2 * PG * (size_t)max_T,
                       st, n, sacs, order, pos, status, max_T, model, prm.max_iter, prm.objective, (double)prm.tol_f,
                       (double)prm.lambda0, (double)prm.box_frac, (double)prm.dt_ms, opc, rmse, mae, iters, dec);
}

hipError_t launch_polish_kernel(const opmm_ctx* ctx, const SacDev* sacs, const int* order, int n, int max_T,
                                const float* pos, const int32_t* status, int model, const opmm_polish_params& prm,
                                float* opc, float* rmse, float* mae, int32_t* iters, int8_t* dec, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (max_T < 1 || max_T > OPMM_MAX_T) return hipErrorInvalidValue;
    switch (polish_group(n, max_T, 4 * opmm_rt::ctx_cu_count(ctx))) {
        case 3: launch_group<3>(sacs, order, n, max_T, pos, status, model, prm, opc, rmse, mae, iters, dec, st); break;
        case 2: launch_group<2>(sacs, order, n, max_T, pos, status, model, prm, opc, rmse, mae, iters, dec, st); break;
        default: launch_group<1>(sacs, order, n, max_T, pos, status, model, prm, opc, rmse, mae, iters, dec, st);
    }
    return hipGetLastError();
}

}  // namespace

namespace opmm_rt {

hipError_t launch_polish(const opmm_ctx* ctx, const SacDev* sacs, int n, int max_T, const float* pos,
                         const int32_t* status, int model, const opmm_polish_params& prm, float* opc, float* rmse,
                         float* mae, hipStream_t st)
{
    return launch_polish_kernel(ctx, sacs, nullptr, n, max_T, pos, status, model, prm, opc, rmse, mae, nullptr,
                                nullptr, st);
}

}  // namespace opmm_rt

extern "C" {

void opmm_polish_params_default(opmm_polish_params* p)
{
    if (!p) return;
    p->max_iter = 20;
    p->objective = OPMM_OBJ_RMSE;
    p->tol_f = 1e-10f;
    p->lambda0 = 1e-3f;
    p->box_frac = 0.25f;
    p->dt_ms = 1.0f;
}

int opmm_sensitivity(opmm_ctx* ctx, const opmm_saccade* sacs, int32_t S, const float* opc, float dt_ms,
                     double* theta_out, double* jac_out, void* stream)
{
    if (!ctx) return OPMM_EINVAL;
    if (S < 0 || (S > 0 && (!sacs || !opc || !theta_out || !jac_out)) || !(dt_ms > 0 && dt_ms <= 1))
        return opmm_rt::fail(ctx, OPMM_EINVAL, "bad sensitivity arguments");
    if (S == 0) return OPMM_OK;
    std::vector<SacDev> hs(S);
    std::vector<int64_t> off(S);
    int64_t acc = 0;
    for (int i = 0; i < S; ++i) {
        if (sacs[i].T < 1 || sacs[i].T > OPMM_MAX_T || !std::isfinite(sacs[i].amp_deg) ||
            !(sacs[i].dur_ms > 0))
            return opmm_rt::fail(ctx, OPMM_EINVAL, "bad saccade record " + std::to_string(i));
        hs[i] = opmm_rt::make_record(sacs[i], 1);
        off[i] = acc;
        acc += sacs[i].T;
    }
    hipStream_t st = (hipStream_t)stream;
    SacDev* d_sacs = nullptr;
    int64_t* d_off = nullptr;
    int rc = OPMM_OK;
    auto ok = [&](hipError_t e, const char* w) { if (rc == OPMM_OK && e != hipSuccess) rc = opmm_rt::hip_fail(ctx, e, w); };
    ok(hipMallocAsync((void**)&d_sacs, sizeof(SacDev) * S, st), "alloc");
    ok(hipMallocAsync((void**)&d_off, sizeof(int64_t) * S, st), "alloc");
    ok(hipMemcpyAsync(d_sacs, hs.data(), sizeof(SacDev) * S, hipMemcpyHostToDevice, st), "copy");
    ok(hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * S, hipMemcpyHostToDevice, st), "copy");
    if (rc == OPMM_OK) {
        hipLaunchKernelGGL(sensitivity_kernel, dim3(S), dim3(64), 0, st, S, d_sacs, d_off, opc, (double)dt_ms,
                           theta_out, jac_out);
        ok(hipGetLastError(), "sensitivity_kernel");
    }
    // the host arrays are released when this call returns: wait for the copies
    ok(hipStreamSynchronize(st), "sync");
    if (d_sacs) (void)hipFreeAsync(d_sacs, st);
    if (d_off) (void)hipFreeAsync(d_off, st);
    return rc;
}

int opmm_polish(opmm_ctx* ctx, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                const opmm_polish_params* prm, int32_t model, float* opc_inout, float* rmse_out, float* mae_out,
                int32_t* iters_out, int8_t* decisions_out, void* stream)
{
    if (!ctx) return OPMM_EINVAL;
    if (!prm || prm->max_iter < 0 || prm->max_iter > 10000 ||
        (prm->objective != OPMM_OBJ_RMSE && prm->objective != OPMM_OBJ_MAE) || !(prm->tol_f >= 0) ||
        !(prm->lambda0 > 0) || !(prm->box_frac > 0 && prm->box_frac < 1) || !(prm->dt_ms > 0 && prm->dt_ms <= 1) ||
        (model != 9 && model != 18))
        return opmm_rt::fail(ctx, OPMM_EINVAL, "bad polish parameters");
    if (S < 0 || (S > 0 && (!pos || !sacs || !opc_inout || !rmse_out)))
        return opmm_rt::fail(ctx, OPMM_EINVAL, "bad arguments");
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
    hipError_t e = launch_polish_kernel(ctx, d_sacs, opmm_rt::batch_order(ctx), S, max_T, pos, status, (int)model,
                                        *prm, opc_inout, rmse_out, mae_out, iters_out, decisions_out, st);
    if (e != hipSuccess) return opmm_rt::hip_fail(ctx, e, "polish_kernel");
    return OPMM_OK;
}

}  // extern "C"
