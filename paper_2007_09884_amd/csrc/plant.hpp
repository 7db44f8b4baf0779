// Device-side model of the 18-parameter oculomotor plant (arXiv 2007.09884,
// Section 2.1 and Section 2.2.1 / Table 1) for one candidate per lane.
//
// Units: time in ms (viscosities scaled by 1e3, inertia by 1e6 from Table 1's
// second-based units), angles in degrees, forces in grams.
//
// State x = (theta, omega, x_ag, x_ant, F_ag, F_ant).  The plant is linear and
// time-invariant on each piece of the pulse-step control (pulse on [0, PW)
// with the activation time constants, step afterwards with the deactivation
// time constants), so one sample period dt advances the deviation from the
// piece's equilibrium by a fixed matrix: d_{k+1} = Phi d_k.  Phi = exp(A dt) is
// formed once per candidate in "D-form" (D = Phi - I, Taylor polynomial by
// Horner's rule, then squarings): storing Phi - I keeps the slow modes
// (|1 - mu| ~ 0.02 per ms) at full relative precision.  The recurrence type R
// is FP64 by default (FP32 stays buildable); candidates are FP32.  The sample
// that contains the pulse end is split exactly at PW with two Taylor
// exponential-vector products.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace opmm {

constexpr int P = 18;

// Precision of the per-sample recurrence and of the transition matrix.
#ifndef OPMM_REC_T
#define OPMM_REC_T double
#endif
using R = OPMM_REC_T;

__device__ __forceinline__ float fmr(float a, float b, float c) { return __fmaf_rn(a, b, c); }
__device__ __forceinline__ double fmr(double a, double b, double c) { return __fma_rn(a, b, c); }

// Taylor degree and squarings of the one-sample transition, and the degree of
// the exponential-vector product of the split sample, per precision: each
// set puts the truncation error below that precision's rounding floor over
// +/-25% boxes (FP64: ~5e-9 deg on 150-sample traces; FP32: the RMSE of a
// candidate stays within ~8e-6 deg of its FP64 value with degrees 7 and 6,
// as with 8 and 8, while a degree-6 transition doubles that).
// The scalar setup (matrix entries, equilibria) and the squared-residual sum
// run in FP64 for the FP64 recurrence; the FP32 recurrence screens candidates
// only, so its setup and sum stay in FP32 (the FP32 rate is twice the FP64
// rate on this chip) and their rounding joins the screening error budget.
#ifndef OPMM_F32_TAYLOR_M
#define OPMM_F32_TAYLOR_M 7
#endif
#ifndef OPMM_F32_EXPMV_M
#define OPMM_F32_EXPMV_M 6
#endif
template <class RT>
struct Prec {
    static constexpr int taylor_m = sizeof(RT) == 8 ? 6 : OPMM_F32_TAYLOR_M;
    static constexpr int taylor_sq = sizeof(RT) == 8 ? 2 : 0;
    static constexpr int expmv_m = sizeof(RT) == 8 ? 11 : OPMM_F32_EXPMV_M;
    using scalar = RT;  // type of plant_scalars
    using acc = RT;     // type of the squared-residual sum
};

// Table 1 nominal values, in the table's order and units.  The pulse width
// (index 17) is the saccade duration minus 6 ms.
__host__ __device__ inline float nominal_param(int j, float dur_ms)
{
    switch (j) {
    case 0: return 2.5f;       // K_SE_AG
    case 1: return 2.5f;       // K_SE_ANT
    case 2: return 1.2f;       // K_LT_AG
    case 3: return 1.2f;       // K_LT_ANT
    case 4: return 0.046f;     // B_AG
    case 5: return 0.022f;     // B_ANT
    case 6: return 0.06f;      // B_P
    case 7: return 0.8f;       // N_C_AG
    case 8: return 0.5f;       // N_C_ANT
    case 9: return 0.000043f;  // J
    case 10: return 11.7f;     // tau_AC_AG
    case 11: return 2.4f;      // tau_AC_ANT
    case 12: return 2.0f;      // tau_DE_AG
    case 13: return 1.9f;      // tau_DE_ANT
    case 14: return 14.0f;     // N_C_FIX
    case 15: return 55.0f;     // N_SAC_AG
    case 16: return 0.5f;      // N_SAC_ANT
    default: return dur_ms - 6.0f; // PW
    }
}

// Table 1 in FP64 (the decimal values as printed), for methods whose iterates
// live in FP64 relative to nominal.
__host__ __device__ inline double nominal_param_f64(int j, double dur_ms)
{
    switch (j) {
    case 0: return 2.5;
    case 1: return 2.5;
    case 2: return 1.2;
    case 3: return 1.2;
    case 4: return 0.046;
    case 5: return 0.022;
    case 6: return 0.06;
    case 7: return 0.8;
    case 8: return 0.5;
    case 9: return 0.000043;
    case 10: return 11.7;
    case 11: return 2.4;
    case 12: return 2.0;
    case 13: return 1.9;
    case 14: return 14.0;
    case 15: return 55.0;
    case 16: return 0.5;
    default: return dur_ms - 6.0;
    }
}

// ---------------------------------------------------------------------------
// Candidate stream
// ---------------------------------------------------------------------------

// SplitMix64 (Steele, Lea & Flood 2014): output n of the generator seeded
// with `seed` is mix(seed + n * golden_gamma).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t stream_counter(uint32_t round, uint32_t idx, uint32_t k)
{
    return 1ull + (((uint64_t)round << 36) | ((uint64_t)idx << 4) | (uint64_t)k);
}

// 24-bit uniform u -> s = u/2^23 - 1 (exact) -> clamp(fma(w, s, c)).
__device__ __forceinline__ float box_draw(uint32_t u, float c, float w, float lo, float hi)
{
    float s = __fmaf_rn((float)u, 0x1p-23f, -1.0f);
    float v = __fmaf_rn(w, s, c);
    return __builtin_amdgcn_fmed3f(v, lo, hi);  // = clamp to [lo, hi] (lo <= hi, v finite)
}

struct Box {
    float c[P], w[P], lo[P], hi[P];
};

// The 9-parameter model (Table 2) shares one series elasticity and one
// length-tension value between the muscles.
__host__ __device__ inline bool fixed_in_model9(int j) { return (j >= 10 && j <= 13) || j >= 15; }

// Full candidate `idx` of round `round` (index 0 is the centre).
__device__ __forceinline__ void draw_candidate(uint64_t seed, uint32_t round, uint32_t idx,
                                               const Box& b, float p[P], int model = 18)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        uint64_t z = splitmix64(seed, stream_counter(round, idx, k));
        uint32_t ua = (uint32_t)(z >> 40);
        uint32_t ub = (uint32_t)(z >> 16) & 0xFFFFFFu;
        p[2 * k] = box_draw(ua, b.c[2 * k], b.w[2 * k], b.lo[2 * k], b.hi[2 * k]);
        p[2 * k + 1] = box_draw(ub, b.c[2 * k + 1], b.w[2 * k + 1], b.lo[2 * k + 1], b.hi[2 * k + 1]);
    }
    if (idx == 0) {
#pragma unroll
        for (int j = 0; j < P; ++j) p[j] = b.c[j];
    }
    if (model == 9) {
        p[1] = p[0];
        p[3] = p[2];
    }
}

// Only the pulse width of candidate idx (last draw, low half).
__device__ __forceinline__ float draw_pw(uint64_t seed, uint32_t round, uint32_t idx, const Box& b)
{
    uint64_t z = splitmix64(seed, stream_counter(round, idx, 8));
    uint32_t ub = (uint32_t)(z >> 16) & 0xFFFFFFu;
    float v = box_draw(ub, b.c[17], b.w[17], b.lo[17], b.hi[17]);
    return idx == 0 ? b.c[17] : v;
}

// ---------------------------------------------------------------------------
// Plant coefficients of one candidate
// ---------------------------------------------------------------------------

template <class RT>
struct PlantT {
    // continuous-time system matrix entries (per ms); theta' = omega is implicit
    RT a10, a11, a12, a13;      // omega row: theta, omega, x_ag, x_ant
    RT a20, a22, g2;            // x_ag row: theta, x_ag, F_ag
    RT a30, a33, g3;            // x_ant row: theta, x_ant, F_ant
    RT q1a, q1n, q2a, q2n;      // F rows: -1/tau, pulse (activation) and post (deactivation)
    // one-sample transition in D-form (Phi - I)
    RT m[4][4];                 // mechanical block
    RT x1[4][2], x2[4][2];      // coupling to (F_ag, F_ant), pulse and post pieces
    RT e1[2], e2[2];            // F decay factor minus one, pulse and post pieces
    // equilibria and switching
    RT th1;                     // theta at the pulse equilibrium
    RT amp;                     // theta at the post equilibrium (= amplitude)
    RT sh[6];                   // pulse equilibrium minus post equilibrium
    RT d0[6];                   // resting state minus pulse equilibrium
    float pw;                  // PW (ms)
    double pwd;                // PW in sample periods
};
using Plant = PlantT<R>;

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// 1/x in FP64: hardware reciprocal refined by two Newton steps (the relative
// error of the seed squares each step), within an ulp or two of the rounded quotient.
__device__ __forceinline__ double rcp64(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = __fma_rn(-x, y, 1.0);
    y = __fma_rn(y, e, y);
    e = __fma_rn(-x, y, 1.0);
    return __fma_rn(y, e, y);
}
// The FP32 counterpart for plant_scalars<float>: one Newton step on the hardware reciprocal.
__device__ __forceinline__ float rcp64(float x)
{
    float y = rcp(x);
    return __fmaf_rn(y, __fmaf_rn(-x, y, 1.0f), y);
}

// Type of the decimal constants in plant_scalars: the scalar itself for plain
// types, FP64 for the dual numbers of the sensitivity pass.
template <class S> struct LitT { using type = double; };
template <> struct LitT<float> { using type = float; };

// mechanical rows of (s*A) V, plus `acc` on the diagonal of column `diag` (-1: none)
#define OPMM_MV(s10, s11, s12, s13, s20, s22, s30, s33, sv, V0, V1, V2, V3, o0, o1, o2, o3, i0, i1, i2, i3) \
    do {                                                                                               \
        o0 = fmr(sv, V1, i0);                                                                    \
        o1 = fmr(s13, V3, fmr(s12, V2, fmr(s11, V1, fmr(s10, V0, i1))));       \
        o2 = fmr(s22, V2, fmr(s20, V0, i2));                                               \
        o3 = fmr(s33, V3, fmr(s30, V0, i3));                                               \
    } while (0)

// Horner evaluation of D = sum_{k=1..M} (hA)^k / k! for the augmented block
// matrix [[Mech, G1, G2], [0, Q1, 0], [0, 0, Q2]] whose off-diagonal blocks
// give the pulse-piece and post-piece coupling columns at once, on the step
// h/2^SQ, then SQ squarings in D-form: D_2h = D_h^2 + 2 D_h.  The Horner
// iterates P_k = I + (B/k) P_{k+1} (B = hA) are carried scaled, Q_k = c_k P_k
// with c_M = M and c_k = k c_{k+1}: then Q_M = M I + B, Q_k = c_k I + B Q_{k+1}
// and D = B Q_2 / M!, so the entries of B are formed once instead of once per
// step (fewer instructions and fewer live registers).
template <class RT>
__device__ __forceinline__ void transition_dform(PlantT<RT>& pl, RT hfull)
{
    constexpr int M = Prec<RT>::taylor_m, SQ = Prec<RT>::taylor_sq;
    const RT h = hfull * (RT(1) / RT(1 << SQ));
    const RT qv[4] = {pl.q1a, pl.q1n, pl.q2a, pl.q2n};
    const RT s10 = pl.a10 * h, s11 = pl.a11 * h, s12 = pl.a12 * h, s13 = pl.a13 * h;
    const RT s20 = pl.a20 * h, s22 = pl.a22 * h, s30 = pl.a30 * h, s33 = pl.a33 * h;
    const RT sg2 = pl.g2 * h, sg3 = pl.g3 * h;
    RT sq[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) sq[c] = qv[c] * h;
    RT pm[4][4], px[4][4], pd[4];
    {   // Q_M = M I + B
        const RT m = RT(M);
        pm[0][0] = m;   pm[0][1] = h;      pm[0][2] = RT(0);    pm[0][3] = RT(0);
        pm[1][0] = s10; pm[1][1] = m + s11; pm[1][2] = s12;     pm[1][3] = s13;
        pm[2][0] = s20; pm[2][1] = RT(0);  pm[2][2] = m + s22;  pm[2][3] = RT(0);
        pm[3][0] = s30; pm[3][1] = RT(0);  pm[3][2] = RT(0);    pm[3][3] = m + s33;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            px[0][c] = RT(0); px[1][c] = RT(0);
            px[2][c] = (c & 1) ? RT(0) : sg2;
            px[3][c] = (c & 1) ? sg3 : RT(0);
            pd[c] = m + sq[c];
        }
    }
    RT ck = RT(M);
#pragma unroll
    for (int k = M - 1; k >= 1; --k) {
        // k >= 2: Q_k = c_k I + B Q_{k+1};  k == 1: D = (B / M!) Q_2
        RT one, t10, t11, t12, t13, t20, t22, t30, t33, tv, tg2, tg3, tq[4];
        if (k >= 2) {
            ck = ck * RT(k);
            one = ck;
            t10 = s10; t11 = s11; t12 = s12; t13 = s13; t20 = s20; t22 = s22; t30 = s30; t33 = s33;
            tv = h; tg2 = sg2; tg3 = sg3;
#pragma unroll
            for (int c = 0; c < 4; ++c) tq[c] = sq[c];
        } else {
            const RT f = RT(1) / ck;  // 1 / M!, rounded once
            one = RT(0);
            t10 = s10 * f; t11 = s11 * f; t12 = s12 * f; t13 = s13 * f;
            t20 = s20 * f; t22 = s22 * f; t30 = s30 * f; t33 = s33 * f;
            tv = h * f; tg2 = sg2 * f; tg3 = sg3 * f;
#pragma unroll
            for (int c = 0; c < 4; ++c) tq[c] = sq[c] * f;
        }
        RT nm[4][4], nx[4][4], nd[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            OPMM_MV(t10, t11, t12, t13, t20, t22, t30, t33, tv, pm[0][c], pm[1][c], pm[2][c], pm[3][c],
                    nm[0][c], nm[1][c], nm[2][c], nm[3][c],
                    c == 0 ? one : RT(0), c == 1 ? one : RT(0), c == 2 ? one : RT(0), c == 3 ? one : RT(0));
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const RT ga = (c & 1) ? RT(0) : tg2 * pd[c];
            const RT gn = (c & 1) ? tg3 * pd[c] : RT(0);
            OPMM_MV(t10, t11, t12, t13, t20, t22, t30, t33, tv, px[0][c], px[1][c], px[2][c], px[3][c],
                    nx[0][c], nx[1][c], nx[2][c], nx[3][c], RT(0), RT(0), ga, gn);
            nd[c] = fmr(tq[c], pd[c], one);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int c = 0; c < 4; ++c) { pm[i][c] = nm[i][c]; px[i][c] = nx[i][c]; }
            pd[i] = nd[i];
        }
    }
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
        RT nm[4][4], nx[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                RT a = pm[i][c] + pm[i][c];
#pragma unroll
                for (int k = 0; k < 4; ++k) a = fmr(pm[i][k], pm[k][c], a);
                nm[i][c] = a;
                RT b = px[i][c] * (pd[c] + RT(2));
#pragma unroll
                for (int k = 0; k < 4; ++k) b = fmr(pm[i][k], px[k][c], b);
                nx[i][c] = b;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int c = 0; c < 4; ++c) { pm[i][c] = nm[i][c]; px[i][c] = nx[i][c]; }
            pd[i] = pd[i] * (pd[i] + RT(2));
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int c = 0; c < 4; ++c) pl.m[i][c] = pm[i][c];
        pl.x1[i][0] = px[i][0]; pl.x1[i][1] = px[i][1];
        pl.x2[i][0] = px[i][2]; pl.x2[i][1] = px[i][3];
    }
    pl.e1[0] = pd[0]; pl.e1[1] = pd[1];
    pl.e2[0] = pd[2]; pl.e2[1] = pd[3];
}


// Continuous-time coefficients (per ms) and the statics of candidate p for a
// saccade of amplitude amp (deg): the matrix entries of the mechanical block,
// the force couplings and active-state rates of both pieces, the pulse
// equilibrium's theta, and the deviations rest - pulse equilibrium and pulse
// equilibrium - post equilibrium (Section 2.1).  Generic in the scalar so that
// the sensitivity pass runs the very same formulas on dual numbers.
template <class S>
struct PlantScalars {
    S a10, a11, a12, a13, a20, a22, g2, a30, a33, g3;
    S q1a, q1n, q2a, q2n;
    S th1;
    S d0[6];
    S sh[6];
};

template <class S>
__device__ __forceinline__ void plant_scalars(const S p[P], S amp, PlantScalars<S>& o)
{
    using L = typename LitT<S>::type;
    const S kse_a = p[0], kse_n = p[1], klt_a = p[2], klt_n = p[3];
    const S b_a = p[4] * L(1e3), b_n = p[5] * L(1e3), b_p = p[6] * L(1e3);
    const S nc_a = p[7], nc_n = p[8];
    const S kp = nc_a + nc_n;            // passive elasticity = sum of tension slopes
    const S jm = p[9] * L(1e6);
    const S ij = rcp64(jm), iba = rcp64(b_a), ibn = rcp64(b_n);
    o.a10 = -(kse_a + kse_n + kp) * ij;
    o.a11 = -b_p * ij;
    o.a12 = kse_a * ij;
    o.a13 = -kse_n * ij;
    o.a20 = kse_a * iba;
    o.a22 = -(klt_a + kse_a) * iba;
    o.g2 = iba;
    o.a30 = -kse_n * ibn;
    o.a33 = -(klt_n + kse_n) * ibn;
    o.g3 = ibn;
    o.q1a = -rcp64(p[10]);
    o.q1n = -rcp64(p[11]);
    o.q2a = -rcp64(p[12]);
    o.q2n = -rcp64(p[13]);

    // statics: c_m = K_SE/(K_SE + K_LT) is the share of the active state the series element carries
    const S iksa = rcp64(kse_a), iksn = rcp64(kse_n);
    const S ica = L(1.0) + klt_a * iksa, icn = L(1.0) + klt_n * iksn;  // 1/c_m
    const S ca = kse_a * rcp64(kse_a + klt_a), cn = kse_n * rcp64(kse_n + klt_n);
    const S kt = kp + ca * klt_a + cn * klt_n;
    const S nfix = p[14], ns_a = p[15], ns_n = p[16], a = amp;
    // rest: theta = 0, fixation tension N_C_FIX on both muscles
    const S xa0 = nfix * iksa, xn0 = nfix * iksn;
    const S fa0 = nfix * ica, fn0 = nfix * icn;
    // pulse piece equilibrium (active states at the pulse heights)
    const S th1 = (ca * ns_a - cn * ns_n) * rcp64(kt);
    const S ta1 = ca * (ns_a - klt_a * th1), tn1 = cn * (ns_n + klt_n * th1);
    const S xa1 = th1 + ta1 * iksa, xn1 = tn1 * iksn - th1;
    // post piece equilibrium: the step holds the eye at the amplitude
    const S ta2 = nfix + nc_a * a, tn2 = nfix - nc_n * a;
    const S xa2 = a + ta2 * iksa, xn2 = tn2 * iksn - a;
    const S fa2 = ta2 * ica + klt_a * a, fn2 = tn2 * icn - klt_n * a;
    o.th1 = th1;
    o.d0[0] = -th1; o.d0[1] = S(0.0); o.d0[2] = xa0 - xa1; o.d0[3] = xn0 - xn1;
    o.d0[4] = fa0 - ns_a; o.d0[5] = fn0 - ns_n;
    o.sh[0] = th1 - a; o.sh[1] = S(0.0); o.sh[2] = xa1 - xa2; o.sh[3] = xn1 - xn2;
    o.sh[4] = ns_a - fa2; o.sh[5] = ns_n - fn2;
}

// Coefficients, transition and equilibria of candidate p for a saccade of
// amplitude amp (deg), sample period dt (ms).  The scalar part is formed in ST
// and rounded once to RT.  FP32 chains of reciprocals shift the equilibria by
// a few ulps of ~10 deg, i.e. ~1e-6 deg on every sample: below the FP32
// recurrence's own error, and a bias the FP64 recurrence does not take.
template <class RT, class ST = typename Prec<RT>::scalar>
__device__ __forceinline__ void plant_setup(const float p[P], float amp, float dt, PlantT<RT>& pl)
{
    ST pd[P];
#pragma unroll
    for (int j = 0; j < P; ++j) pd[j] = p[j];
    PlantScalars<ST> c;
    plant_scalars(pd, (ST)amp, c);
    pl.a10 = (RT)c.a10; pl.a11 = (RT)c.a11; pl.a12 = (RT)c.a12; pl.a13 = (RT)c.a13;
    pl.a20 = (RT)c.a20; pl.a22 = (RT)c.a22; pl.g2 = (RT)c.g2;
    pl.a30 = (RT)c.a30; pl.a33 = (RT)c.a33; pl.g3 = (RT)c.g3;
    pl.q1a = (RT)c.q1a; pl.q1n = (RT)c.q1n; pl.q2a = (RT)c.q2a; pl.q2n = (RT)c.q2n;
    transition_dform(pl, (RT)dt);
    pl.th1 = (RT)c.th1;
    pl.amp = amp;
#pragma unroll
    for (int i = 0; i < 6; ++i) { pl.d0[i] = (RT)c.d0[i]; pl.sh[i] = (RT)c.sh[i]; }
    pl.pw = p[17];
    pl.pwd = (double)p[17] * rcp64((double)dt);
}

// d <- Phi d for one sample (D-form: d + D d)
template <class RT>
__device__ __forceinline__ void step(const PlantT<RT>& pl, const RT (&x)[4][2], const RT (&e)[2], RT d[6])
{
    RT n[4];
    // the row's own state is the addend of the first fma
    n[0] = fmr(pl.m[0][0], d[0], d[0]);
    n[1] = fmr(pl.m[1][1], d[1], d[1]);
    n[2] = fmr(pl.m[2][2], d[2], d[2]);
    n[3] = fmr(pl.m[3][3], d[3], d[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c != i) n[i] = fmr(pl.m[i][c], d[c], n[i]);
        n[i] = fmr(x[i][0], d[4], n[i]);
        n[i] = fmr(x[i][1], d[5], n[i]);
    }
    d[4] = fmr(e[0], d[4], d[4]);
    d[5] = fmr(e[1], d[5], d[5]);
#pragma unroll
    for (int i = 0; i < 4; ++i) d[i] = n[i];
}

// v <- exp(A t) v by a Taylor polynomial (degree Prec::expmv_m) in Horner form (t <= dt).
template <class RT>
__device__ __forceinline__ void expmv(const PlantT<RT>& pl, RT qa, RT qn, RT t, RT v[6])
{
    RT w[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) w[i] = v[i];
#pragma unroll
    for (int k = Prec<RT>::expmv_m; k >= 1; --k) {
        RT s = t * (RT(1) / RT(k));
        asm volatile("" : "+v"(s));
        RT aw[6];
        aw[0] = w[1];
        aw[1] = fmr(pl.a13, w[3], fmr(pl.a12, w[2], fmr(pl.a11, w[1], pl.a10 * w[0])));
        aw[2] = fmr(pl.g2, w[4], fmr(pl.a22, w[2], pl.a20 * w[0]));
        aw[3] = fmr(pl.g3, w[5], fmr(pl.a33, w[3], pl.a30 * w[0]));
        aw[4] = qa * w[4];
        aw[5] = qn * w[5];
#pragma unroll
        for (int i = 0; i < 6; ++i) w[i] = fmr(s, aw[i], v[i]);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = w[i];
}

// The sample that contains the pulse end: pulse dynamics for frac*dt, switch
// to the post piece's coordinates, post dynamics for the rest of the sample.
template <class RT>
__device__ __forceinline__ void split_step(const PlantT<RT>& pl, RT frac, RT dt, RT d[6])
{
    expmv(pl, pl.q1a, pl.q1n, frac * dt, d);
#pragma unroll
    for (int i = 0; i < 6; ++i) d[i] += pl.sh[i];
    expmv(pl, pl.q2a, pl.q2n, (RT(1) - frac) * dt, d);
}

// wave-wide min / max of an int (64 lanes)
__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Integer sample index that holds the pulse end (-1: no pulse), clamped to
// [-1, T], and the fraction of that sample spent in the pulse.
template <class RT>
__device__ __forceinline__ int pulse_end_sample(double pw, int T, RT& frac)
{
    double fl = floor(pw);
    int k0;
    if (!(pw > 0.0)) { k0 = -1; frac = RT(0); }
    else if (fl >= (double)T) { k0 = T; frac = RT(0); }
    else { k0 = (int)fl; frac = (RT)(pw - fl); }
    return k0;
}

// Run the trajectory theta_k, k = 0..T-1, calling sink(k, dtheta, theta_eq)
// with theta_k = dtheta + theta_eq.  kmin/kmax: wave-uniform bounds of the
// lanes' pulse-end samples; samples below kmin are pulse for every lane and
// samples above kmax post for every lane, so only [kmin, kmax] branches.
template <int UNROLL, class RT, class Sink>
__device__ __forceinline__ void run_trajectory(const PlantT<RT>& pl, int T, RT dt, int k0, RT frac,
                                               int kmin, int kmax, Sink& sink)
{
    RT d[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) d[i] = pl.d0[i];
    RT theq = pl.th1;
    if (k0 < 0) {  // PW <= 0: no pulse, the step acts from t = 0
#pragma unroll
        for (int i = 0; i < 6; ++i) d[i] += pl.sh[i];
        theq = pl.amp;
    }
    int k = 0;
    const int ka = min(kmin, T);
#pragma unroll UNROLL
    for (; k < ka; ++k) {
        sink(k, d[0], theq);
        step(pl, pl.x1, pl.e1, d);
    }
    const int kb = min(kmax, T - 1);
#pragma unroll 1
    for (; k <= kb; ++k) {
        sink(k, d[0], theq);
        if (k < k0) {
            step(pl, pl.x1, pl.e1, d);
        } else if (k == k0) {
            split_step(pl, frac, dt, d);
            theq = pl.amp;
        } else {
            step(pl, pl.x2, pl.e2, d);
        }
    }
#pragma unroll UNROLL
    for (; k < T; ++k) {
        sink(k, d[0], theq);
        step(pl, pl.x2, pl.e2, d);
    }
}

}  // namespace opmm
