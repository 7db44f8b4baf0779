// Device-side model of the 18-parameter oculomotor plant (arXiv 2007.09884,
// Section 2.1 and Section 2.2.1 / Table 1) for one candidate per lane, FP32.
//
// Units: time in ms (viscosities scaled by 1e3, inertia by 1e6 from Table 1's
// second-based units), angles in degrees, forces in grams.
//
// State x = (theta, omega, x_ag, x_ant, F_ag, F_ant).  The plant is linear and
// time-invariant on each piece of the pulse-step control (pulse on [0, PW)
// with the activation time constants, step afterwards with the deactivation
// time constants), so one sample period dt advances the deviation from the
// piece's equilibrium by a fixed matrix: d_{k+1} = Phi d_k.  Phi = exp(A dt) is
// formed once per candidate in "D-form" (D = Phi - I, degree-8 Taylor
// polynomial evaluated by Horner's rule): storing Phi - I keeps the slow modes
// (|1 - mu| ~ 0.02 per ms) at full relative precision, which is what lets the
// whole path run in FP32.  The sample that contains the pulse end is split
// exactly at PW with two Taylor exponential-vector products.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace opmm {

constexpr int P = 18;

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
    return fminf(fmaxf(v, lo), hi);
}

struct Box {
    float c[P], w[P], lo[P], hi[P];
};

// Full candidate `idx` of round `round` (index 0 is the centre).
__device__ __forceinline__ void draw_candidate(uint64_t seed, uint32_t round, uint32_t idx,
                                               const Box& b, float p[P])
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

struct Plant {
    // continuous-time system matrix entries (per ms); theta' = omega is implicit
    float a10, a11, a12, a13;  // omega row: theta, omega, x_ag, x_ant
    float a20, a22, g2;        // x_ag row: theta, x_ag, F_ag
    float a30, a33, g3;        // x_ant row: theta, x_ant, F_ant
    float q1a, q1n, q2a, q2n;  // F rows: -1/tau, pulse (activation) and post (deactivation)
    // one-sample transition in D-form (Phi - I)
    float m[4][4];             // mechanical block
    float x1[4][2], x2[4][2];  // coupling to (F_ag, F_ant), pulse and post pieces
    float e1[2], e2[2];        // F decay factor minus one, pulse and post pieces
    // equilibria and switching
    float th1;                 // theta at the pulse equilibrium
    float amp;                 // theta at the post equilibrium (= amplitude)
    float sh[6];               // pulse equilibrium minus post equilibrium
    float d0[6];               // resting state minus pulse equilibrium
    float pw;                  // PW in sample periods
};

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// mechanical rows of (s*A) V, plus `acc` on the diagonal of column `diag` (-1: none)
#define OPMM_MV(s10, s11, s12, s13, s20, s22, s30, s33, sv, V0, V1, V2, V3, o0, o1, o2, o3, i0, i1, i2, i3) \
    do {                                                                                               \
        o0 = __fmaf_rn(sv, V1, i0);                                                                    \
        o1 = __fmaf_rn(s13, V3, __fmaf_rn(s12, V2, __fmaf_rn(s11, V1, __fmaf_rn(s10, V0, i1))));       \
        o2 = __fmaf_rn(s22, V2, __fmaf_rn(s20, V0, i2));                                               \
        o3 = __fmaf_rn(s33, V3, __fmaf_rn(s30, V0, i3));                                               \
    } while (0)

// Horner evaluation of D = sum_{k=1..8} (hA)^k / k! for the augmented block
// matrix [[Mech, G1, G2], [0, Q1, 0], [0, 0, Q2]] whose off-diagonal blocks
// give the pulse-piece and post-piece coupling columns at once.
__device__ __forceinline__ void transition_dform(Plant& pl, float h)
{
    constexpr int M = 8;
    float pm[4][4], px[4][4], pd[4];
    const float qv[4] = {pl.q1a, pl.q1n, pl.q2a, pl.q2n};
    {   // P_M = I + hA/M
        const float s = h * (1.0f / M);
        const float s10 = pl.a10 * s, s11 = pl.a11 * s, s12 = pl.a12 * s, s13 = pl.a13 * s;
        const float s20 = pl.a20 * s, s22 = pl.a22 * s, s30 = pl.a30 * s, s33 = pl.a33 * s;
        pm[0][0] = 1.0f; pm[0][1] = s;    pm[0][2] = 0.0f; pm[0][3] = 0.0f;
        pm[1][0] = s10;  pm[1][1] = 1.0f + s11; pm[1][2] = s12; pm[1][3] = s13;
        pm[2][0] = s20;  pm[2][1] = 0.0f; pm[2][2] = 1.0f + s22; pm[2][3] = 0.0f;
        pm[3][0] = s30;  pm[3][1] = 0.0f; pm[3][2] = 0.0f; pm[3][3] = 1.0f + s33;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            px[0][c] = 0.0f; px[1][c] = 0.0f;
            px[2][c] = (c & 1) ? 0.0f : pl.g2 * s;
            px[3][c] = (c & 1) ? pl.g3 * s : 0.0f;
            pd[c] = __fmaf_rn(qv[c], s, 1.0f);
        }
    }
#pragma unroll
    for (int k = M - 1; k >= 1; --k) {
        // k >= 2: P <- I + (h/k) A P ;  k == 1: D <- h A P
        const float s = (k == 1) ? h : h * (1.0f / k);
        const float one = (k == 1) ? 0.0f : 1.0f;
        const float s10 = pl.a10 * s, s11 = pl.a11 * s, s12 = pl.a12 * s, s13 = pl.a13 * s;
        const float s20 = pl.a20 * s, s22 = pl.a22 * s, s30 = pl.a30 * s, s33 = pl.a33 * s;
        const float sg2 = pl.g2 * s, sg3 = pl.g3 * s;
        float nm[4][4], nx[4][4], nd[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            OPMM_MV(s10, s11, s12, s13, s20, s22, s30, s33, s, pm[0][c], pm[1][c], pm[2][c], pm[3][c],
                    nm[0][c], nm[1][c], nm[2][c], nm[3][c],
                    c == 0 ? one : 0.0f, c == 1 ? one : 0.0f, c == 2 ? one : 0.0f, c == 3 ? one : 0.0f);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float ga = (c & 1) ? 0.0f : sg2 * pd[c];
            const float gn = (c & 1) ? sg3 * pd[c] : 0.0f;
            OPMM_MV(s10, s11, s12, s13, s20, s22, s30, s33, s, px[0][c], px[1][c], px[2][c], px[3][c],
                    nx[0][c], nx[1][c], nx[2][c], nx[3][c], 0.0f, 0.0f, ga, gn);
            nd[c] = __fmaf_rn(qv[c] * s, pd[c], one);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int c = 0; c < 4; ++c) { pm[i][c] = nm[i][c]; px[i][c] = nx[i][c]; }
            pd[i] = nd[i];
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

// Coefficients, transition and equilibria of candidate p for a saccade of
// amplitude amp (deg), sample period dt (ms).
__device__ __forceinline__ void plant_setup(const float p[P], float amp, float dt, Plant& pl)
{
    const float kse_a = p[0], kse_n = p[1], klt_a = p[2], klt_n = p[3];
    const float b_a = p[4] * 1e3f, b_n = p[5] * 1e3f, b_p = p[6] * 1e3f;
    const float nc_a = p[7], nc_n = p[8];
    const float kp = nc_a + nc_n;             // passive elasticity = sum of tension slopes
    const float jm = p[9] * 1e6f;
    const float ij = rcp(jm), iba = rcp(b_a), ibn = rcp(b_n);
    pl.a10 = -(kse_a + kse_n + kp) * ij;
    pl.a11 = -b_p * ij;
    pl.a12 = kse_a * ij;
    pl.a13 = -kse_n * ij;
    pl.a20 = kse_a * iba;
    pl.a22 = -(klt_a + kse_a) * iba;
    pl.g2 = iba;
    pl.a30 = -kse_n * ibn;
    pl.a33 = -(klt_n + kse_n) * ibn;
    pl.g3 = ibn;
    pl.q1a = -rcp(p[10]);
    pl.q1n = -rcp(p[11]);
    pl.q2a = -rcp(p[12]);
    pl.q2n = -rcp(p[13]);
    transition_dform(pl, dt);

    // statics: fraction of the active state carried by the series element
    const float iksa = rcp(kse_a), iksn = rcp(kse_n);
    const float ica = 1.0f + klt_a * iksa, icn = 1.0f + klt_n * iksn;  // 1/c_m
    const float ca = rcp(ica), cn = rcp(icn);
    const float kt = kp + ca * klt_a + cn * klt_n;
    const float nfix = p[14], ns_a = p[15], ns_n = p[16];
    // rest: theta = 0, fixation tensions N_C_FIX on both muscles
    const float xa0 = nfix * iksa, xn0 = nfix * iksn;
    const float fa0 = nfix * ica, fn0 = nfix * icn;
    // pulse piece equilibrium (active states at the pulse heights)
    const float th1 = (ca * ns_a - cn * ns_n) * rcp(kt);
    const float ta1 = ca * (ns_a - klt_a * th1), tn1 = cn * (ns_n + klt_n * th1);
    const float xa1 = th1 + ta1 * iksa, xn1 = tn1 * iksn - th1;
    // post piece equilibrium: the step holds the eye at the amplitude
    const float ta2 = __fmaf_rn(nc_a, amp, nfix), tn2 = __fmaf_rn(-nc_n, amp, nfix);
    const float xa2 = amp + ta2 * iksa, xn2 = tn2 * iksn - amp;
    const float fa2 = __fmaf_rn(ta2, ica, klt_a * amp), fn2 = __fmaf_rn(tn2, icn, -klt_n * amp);
    pl.th1 = th1;
    pl.amp = amp;
    pl.d0[0] = -th1; pl.d0[1] = 0.0f; pl.d0[2] = xa0 - xa1; pl.d0[3] = xn0 - xn1;
    pl.d0[4] = fa0 - ns_a; pl.d0[5] = fn0 - ns_n;
    pl.sh[0] = th1 - amp; pl.sh[1] = 0.0f; pl.sh[2] = xa1 - xa2; pl.sh[3] = xn1 - xn2;
    pl.sh[4] = ns_a - fa2; pl.sh[5] = ns_n - fn2;
    pl.pw = p[17] * rcp(dt);
}

// d <- Phi d for one sample (D-form: d + D d)
__device__ __forceinline__ void step(const Plant& pl, const float (&x)[4][2], const float (&e)[2], float d[6])
{
    float n[4];
    // the row's own state is the addend of the first fma
    n[0] = __fmaf_rn(pl.m[0][0], d[0], d[0]);
    n[1] = __fmaf_rn(pl.m[1][1], d[1], d[1]);
    n[2] = __fmaf_rn(pl.m[2][2], d[2], d[2]);
    n[3] = __fmaf_rn(pl.m[3][3], d[3], d[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c != i) n[i] = __fmaf_rn(pl.m[i][c], d[c], n[i]);
        n[i] = __fmaf_rn(x[i][0], d[4], n[i]);
        n[i] = __fmaf_rn(x[i][1], d[5], n[i]);
    }
    d[4] = __fmaf_rn(e[0], d[4], d[4]);
    d[5] = __fmaf_rn(e[1], d[5], d[5]);
#pragma unroll
    for (int i = 0; i < 4; ++i) d[i] = n[i];
}

// v <- exp(A t) v by a degree-8 Taylor polynomial in Horner form (t <= dt).
__device__ __forceinline__ void expmv(const Plant& pl, float qa, float qn, float t, float v[6])
{
    float w[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) w[i] = v[i];
#pragma unroll
    for (int k = 8; k >= 1; --k) {
        const float s = t * (1.0f / k);
        float aw[6];
        aw[0] = w[1];
        aw[1] = __fmaf_rn(pl.a13, w[3], __fmaf_rn(pl.a12, w[2], __fmaf_rn(pl.a11, w[1], pl.a10 * w[0])));
        aw[2] = __fmaf_rn(pl.g2, w[4], __fmaf_rn(pl.a22, w[2], pl.a20 * w[0]));
        aw[3] = __fmaf_rn(pl.g3, w[5], __fmaf_rn(pl.a33, w[3], pl.a30 * w[0]));
        aw[4] = qa * w[4];
        aw[5] = qn * w[5];
#pragma unroll
        for (int i = 0; i < 6; ++i) w[i] = __fmaf_rn(s, aw[i], v[i]);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = w[i];
}

// The sample that contains the pulse end: pulse dynamics for frac*dt, switch
// to the post piece's coordinates, post dynamics for the rest of the sample.
__device__ __forceinline__ void split_step(const Plant& pl, float frac, float dt, float d[6])
{
    expmv(pl, pl.q1a, pl.q1n, frac * dt, d);
#pragma unroll
    for (int i = 0; i < 6; ++i) d[i] += pl.sh[i];
    expmv(pl, pl.q2a, pl.q2n, (1.0f - frac) * dt, d);
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
__device__ __forceinline__ int pulse_end_sample(float pw, int T, float& frac)
{
    float fl = floorf(pw);
    int k0;
    if (!(pw > 0.0f)) { k0 = -1; frac = 0.0f; }
    else if (fl >= (float)T) { k0 = T; frac = 0.0f; }
    else { k0 = (int)fl; frac = pw - fl; }
    return k0;
}

// Run the trajectory theta_k, k = 0..T-1, calling sink(k, dtheta, theta_eq)
// with theta_k = dtheta + theta_eq.  kmin/kmax: wave-uniform bounds of the
// lanes' pulse-end samples; samples below kmin are pulse for every lane and
// samples above kmax post for every lane, so only [kmin, kmax] branches.
template <int UNROLL, class Sink>
__device__ __forceinline__ void run_trajectory(const Plant& pl, int T, float dt, int k0, float frac,
                                               int kmin, int kmax, Sink& sink)
{
    float d[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) d[i] = pl.d0[i];
    float theq = pl.th1;
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
