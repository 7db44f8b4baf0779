/*
 * OPMM oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, FP64 CPU implementation of what the OPMM estimation path
 * computes, written to be checked by eye against the paper (arXiv 2007.09884,
 * "Parallel Oculomotor Plant Mathematical Model for Large Scale Eye Movement
 * Simulation").  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product library never does, and this file
 * shares no code, header, table or helper with the GPU path.
 *
 * Units here are the paper's Table 1 units: time in seconds for the mechanics
 * (J in g*s^2/deg, B in g*s/deg), time constants and the pulse width in ms as
 * printed, angles in degrees, forces in grams.  (The GPU path works in ms; the
 * two were written independently.)
 *
 * What the paper fixes and what is a reading (each reading is restated at the
 * function that uses it):
 *   - Parameter set, order and nominal values: Section 2.2.1, Table 1.
 *   - Component semantics (series elasticity, length-tension, force-velocity,
 *     tension slope/intercept, inertia, passive viscosity; pulse-step control
 *     with activation at onset and deactivation at offset): Section 2.1.
 *   - The equations themselves are not printed.  The plant below is the
 *     linear homeomorphic reading: 6 states (theta, omega, x_ag, x_ant, F_ag,
 *     F_ant), passive elasticity K_P = N_C_AG + N_C_ANT, step levels that hold
 *     the eye at the fixation before and after the saccade.
 *   - Cost: root-mean-square difference between recorded and simulated
 *     trajectories (mean absolute difference, the paper's OptErr of
 *     Section 3.4, is reported alongside).
 *   - Search: uniform candidates in a box around the centre, argmin, box
 *     halving (the paper's estimator is Nelder-Mead, Section 3.3; the box
 *     search is the build's data-parallel estimator).
 *
 * Integrator: classical fixed-step RK4, nsub substeps per sample, the sample
 * that contains the pulse end split exactly at PW.  Pinned in the tests
 * against the matrix-exponential solution of the piecewise-LTI plant.
 *
 * Contents and what pins each part (tests under tests/):
 *   - plant, controls, integrator, cost: the closed form above, equilibria
 *     and force balance, linearity, the force-scale and time-scale
 *     invariances, the onset derivative, hand-computed costs;
 *   - candidate stream (SplitMix64) and box rule: the generator's published
 *     test vectors, exact rational arithmetic, uniform fill;
 *   - box search and the 9-parameter subspace: truth recovery, monotone
 *     cost, brute force on small grids, ties and fixed components;
 *   - Nelder-Mead (Section 3.3, Algorithm 1): the exit rule, the initial
 *     simplex, every step of several runs against the Lagarias definition
 *     (all five kinds of step occur), descent;
 *   - sensitivities and the Levenberg-Marquardt polish (the gradient method
 *     of Section 5): the gauge null vector, affine columns, the Frechet
 *     derivative of expm, numpy's solve, quadratic convergence, box faces,
 *     stationarity.
 * The I-VT extraction reference is plain Python in __init__.py, pinned on
 * hand-built streams and planted saccades.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define NP 18

/* Table 1 (Section 2.2.1): nominal values in the table's order and units.
 * The pulse width PW has no number in the table: it is the saccade duration
 * minus 6 ms, filled in by oracle_nominal(). */
static const double TABLE1_NOMINAL[17] = {
    2.5,      /* K_SE_AG  series elasticity, agonist (g/deg)        */
    2.5,      /* K_SE_ANT series elasticity, antagonist             */
    1.2,      /* K_LT_AG  length-tension, agonist (g/deg)           */
    1.2,      /* K_LT_ANT length-tension, antagonist                */
    0.046,    /* B_AG     force-velocity, agonist (g s/deg)         */
    0.022,    /* B_ANT    force-velocity, antagonist                */
    0.06,     /* B_P      passive viscosity (g s/deg)               */
    0.8,      /* N_C_AG   tension slope, agonist (g/deg)            */
    0.5,      /* N_C_ANT  tension slope, antagonist                 */
    0.000043, /* J        inertial mass (g s^2/deg)                 */
    11.7,     /* tau_AC_AG  activation time, agonist (ms)           */
    2.4,      /* tau_AC_ANT activation time, antagonist (ms)        */
    2.0,      /* tau_DE_AG  deactivation time, agonist (ms)         */
    1.9,      /* tau_DE_ANT deactivation time, antagonist (ms)      */
    14.0,     /* N_C_FIX  tension intercept (g)                     */
    55.0,     /* N_SAC_AG neural pulse height, agonist (g)          */
    0.5,      /* N_SAC_ANT neural pulse height, antagonist (g)      */
};

void oracle_nominal(double dur_ms, double out[NP])
{
    for (int j = 0; j < 17; ++j) out[j] = TABLE1_NOMINAL[j];
    out[17] = dur_ms - 6.0; /* Table 1: PW = saccade duration - 6 ms */
}

/* ------------------------------------------------------------------------- */
/* Plant                                                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    double kse_ag, kse_ant, klt_ag, klt_ant;
    double b_ag, b_ant, bp, kp, j;
    double tac_ag, tac_ant, tde_ag, tde_ant; /* seconds */
    double pw;                               /* seconds */
} plant_t;

static void plant_from_opc(const double p[NP], plant_t* q)
{
    q->kse_ag = p[0];  q->kse_ant = p[1];
    q->klt_ag = p[2];  q->klt_ant = p[3];
    q->b_ag = p[4];    q->b_ant = p[5];   q->bp = p[6];
    q->kp = p[7] + p[8];        /* passive elasticity: the tension slopes' sum */
    q->j = p[9];
    q->tac_ag = p[10] * 1e-3;  q->tac_ant = p[11] * 1e-3;
    q->tde_ag = p[12] * 1e-3;  q->tde_ant = p[13] * 1e-3;
    q->pw = p[17] * 1e-3;
}

/* Fixation tensions of Section 2.1 ("muscle force at eccentricities at the
 * equilibrium points"): T_AG(th) = N_C_FIX + N_C_AG*th,
 * T_ANT(th) = N_C_FIX - N_C_ANT*th.  The neural step that holds the eye at th
 * adds what the length-tension element and the series element take up:
 * S_AG = T_AG*(K_SE+K_LT)/K_SE + K_LT_AG*th, S_ANT = T_ANT*(K_SE+K_LT)/K_SE - K_LT_ANT*th. */
static void step_levels(const double p[NP], double th, double* s_ag, double* s_ant)
{
    double t_ag = p[14] + p[7] * th;
    double t_ant = p[14] - p[8] * th;
    *s_ag = t_ag * (p[0] + p[2]) / p[0] + p[2] * th;
    *s_ant = t_ant * (p[1] + p[3]) / p[1] - p[3] * th;
}

/* Time derivative of the state x = (theta, omega, x_ag, x_ant, F_ag, F_ant)
 * under constant neural inputs n_ag, n_ant and active-state time constants
 * tau_ag, tau_ant (s).  x_m is the contractile-element shortening of muscle m
 * in degree-equivalents; the series element of the agonist is stretched by
 * x_ag - theta, that of the antagonist by x_ant + theta.
 *   globe:           J w' = K_SE_AG(x_ag - th) - K_SE_ANT(x_ant + th) - B_P w - K_P th
 *   force-velocity:  B_m x_m' = F_m - K_LT_m x_m - (series tension)
 *   active state:    tau_m F_m' = N_m - F_m                                 */
void oracle_rhs(const double p[NP], const double x[6], double n_ag, double n_ant,
                double tau_ag, double tau_ant, double dx[6])
{
    plant_t q;
    plant_from_opc(p, &q);
    double th = x[0], w = x[1], xa = x[2], xn = x[3], fa = x[4], fn = x[5];
    double t_se_ag = q.kse_ag * (xa - th);
    double t_se_ant = q.kse_ant * (xn + th);
    dx[0] = w;
    dx[1] = (t_se_ag - t_se_ant - q.bp * w - q.kp * th) / q.j;
    dx[2] = (fa - q.klt_ag * xa - t_se_ag) / q.b_ag;
    dx[3] = (fn - q.klt_ant * xn - t_se_ant) / q.b_ant;
    dx[4] = (n_ag - fa) / tau_ag;
    dx[5] = (n_ant - fn) / tau_ant;
}

/* Equilibrium of the plant when both active states sit at (f_ag, f_ant):
 * set every derivative to zero and solve the statics in closed form. */
void oracle_equilibrium(const double p[NP], double f_ag, double f_ant, double x[6])
{
    plant_t q;
    plant_from_opc(p, &q);
    double c_ag = q.kse_ag / (q.kse_ag + q.klt_ag);
    double c_ant = q.kse_ant / (q.kse_ant + q.klt_ant);
    double th = (c_ag * f_ag - c_ant * f_ant) / (q.kp + c_ag * q.klt_ag + c_ant * q.klt_ant);
    double t_ag = c_ag * (f_ag - q.klt_ag * th);   /* series tensions */
    double t_ant = c_ant * (f_ant + q.klt_ant * th);
    x[0] = th;
    x[1] = 0.0;
    x[2] = th + t_ag / q.kse_ag;
    x[3] = t_ant / q.kse_ant - th;
    x[4] = f_ag;
    x[5] = f_ant;
}

static void rk4_span(const double p[NP], double x[6], double span, int nsub,
                     double n_ag, double n_ant, double tau_ag, double tau_ant)
{
    double h = span / nsub;
    for (int s = 0; s < nsub; ++s) {
        double k1[6], k2[6], k3[6], k4[6], y[6];
        oracle_rhs(p, x, n_ag, n_ant, tau_ag, tau_ant, k1);
        for (int i = 0; i < 6; ++i) y[i] = x[i] + 0.5 * h * k1[i];
        oracle_rhs(p, y, n_ag, n_ant, tau_ag, tau_ant, k2);
        for (int i = 0; i < 6; ++i) y[i] = x[i] + 0.5 * h * k2[i];
        oracle_rhs(p, y, n_ag, n_ant, tau_ag, tau_ant, k3);
        for (int i = 0; i < 6; ++i) y[i] = x[i] + h * k3[i];
        oracle_rhs(p, y, n_ag, n_ant, tau_ag, tau_ant, k4);
        for (int i = 0; i < 6; ++i) x[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
}

/* Pulse-step simulation with explicit control levels (Section 2.1): the eye
 * rests at the equilibrium of the pre-saccadic levels (pre_ag, pre_ant); the
 * pulse (pul_ag, pul_ant) is on for t in [0, PW) with the activation time
 * constants; from t = PW on the post-saccadic step (post_ag, post_ant) acts
 * with the deactivation time constants.  theta at t_k = k*dt_ms, k < T. */
int oracle_simulate_levels(const double p[NP], const double lv[6], int T, double dt_ms,
                           int nsub, double* theta, double* state_out)
{
    if (T < 0 || !(dt_ms > 0) || nsub < 1) return -1;
    plant_t q;
    plant_from_opc(p, &q);
    double x[6];
    oracle_equilibrium(p, lv[0], lv[1], x);
    double dt = dt_ms * 1e-3;
    for (int k = 0; k < T; ++k) {
        theta[k] = x[0];
        if (state_out) memcpy(state_out + 6 * k, x, sizeof x);
        if (k == T - 1) break;
        double t0 = k * dt, t1 = (k + 1) * dt;
        if (t1 <= q.pw) {
            rk4_span(p, x, dt, nsub, lv[2], lv[3], q.tac_ag, q.tac_ant);
        } else if (t0 >= q.pw) {
            rk4_span(p, x, dt, nsub, lv[4], lv[5], q.tde_ag, q.tde_ant);
        } else { /* the pulse ends inside this sample: split exactly at PW */
            rk4_span(p, x, q.pw - t0, nsub, lv[2], lv[3], q.tac_ag, q.tac_ant);
            rk4_span(p, x, t1 - q.pw, nsub, lv[4], lv[5], q.tde_ag, q.tde_ant);
        }
    }
    return 0;
}

/* The model's own control for a saccade of amplitude amp (deg): the step
 * holds fixation at 0 before and at amp after; the pulse heights are the
 * OPC's N_SAC_AG and N_SAC_ANT. */
void oracle_control_levels(const double p[NP], double amp, double lv[6])
{
    step_levels(p, 0.0, &lv[0], &lv[1]);
    lv[2] = p[15];
    lv[3] = p[16];
    step_levels(p, amp, &lv[4], &lv[5]);
}

int oracle_simulate(const double p[NP], double amp, int T, double dt_ms, int nsub, double* theta)
{
    double lv[6];
    oracle_control_levels(p, amp, lv);
    return oracle_simulate_levels(p, lv, T, dt_ms, nsub, theta, NULL);
}

/* ------------------------------------------------------------------------- */
/* Cost                                                                       */
/* ------------------------------------------------------------------------- */

/* The 1-D plant moves along the saccade direction phi (Section 2.2: either
 * version simulates one-dimensional movement).  With C = 2 the prediction is
 * (theta cos phi, theta sin phi); with C = 1 the single channel is the
 * horizontal one, theta cos phi.  RMSE over all samples and channels; the
 * mean absolute difference (the paper's OptErr) alongside. */
void oracle_cost(const double* theta, const float* pos, int T, int C, double dir_deg,
                 double* rmse, double* mae)
{
    double phi = dir_deg * (M_PI / 180.0);
    double u[2] = {cos(phi), sin(phi)};
    double sq = 0.0, ab = 0.0;
    for (int k = 0; k < T; ++k)
        for (int c = 0; c < C; ++c) {
            double e = (double)pos[k * C + c] - theta[k] * u[c];
            sq += e * e;
            ab += fabs(e);
        }
    double n = (double)T * C;
    double r = sqrt(sq / n);
    if (!(r <= HUGE_VAL)) r = HUGE_VAL; /* NaN ranks last */
    *rmse = r;
    if (mae) *mae = ab / n;
}

/* ------------------------------------------------------------------------- */
/* Candidates                                                                 */
/* ------------------------------------------------------------------------- */

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the n-th output (n >= 1) of
 * the generator seeded with `seed` is mix(seed + n * golden_gamma). */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + n * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Candidate idx of round r for a saccade keyed by seed.  Candidate 0 is the
 * centre itself.  Otherwise draw k (k = 0..8) is SplitMix64 output number
 * 1 + (r << 36 | idx << 4 | k); its top 24 bits give parameter 2k and the next
 * 24 bits parameter 2k+1.  A 24-bit draw u maps to s = u/2^23 - 1 in [-1, 1)
 * (exact in FP32), the parameter is fma(w, s, c) rounded once to FP32 and then
 * clamped to the search box [lo, hi]. */
void oracle_candidate(uint64_t seed, uint32_t round, uint32_t idx, const float c[NP],
                      const float w[NP], const float lo[NP], const float hi[NP], float out[NP])
{
    if (idx == 0) {
        memcpy(out, c, NP * sizeof(float));
        return;
    }
    for (int k = 0; k < 9; ++k) {
        uint64_t n = 1 + (((uint64_t)round << 36) | ((uint64_t)idx << 4) | (uint64_t)k);
        uint64_t z = oracle_splitmix64(seed, n);
        uint32_t ua = (uint32_t)(z >> 40);
        uint32_t ub = (uint32_t)((z >> 16) & 0xFFFFFFu);
        uint32_t us[2] = {ua, ub};
        for (int h = 0; h < 2; ++h) {
            int j = 2 * k + h;
            float s = (float)us[h] * 0x1p-23f - 1.0f;
            float v = fmaf(w[j], s, c[j]);
            if (v < lo[j]) v = lo[j];
            if (v > hi[j]) v = hi[j];
            out[j] = v;
        }
    }
}

/* The 9-parameter OPMM (Section 2.2.2, Table 2): one series elasticity and
 * one length-tension value for both muscles, the viscosities, tension slopes,
 * inertia and tension intercept free; the neuronal-control parameters (the
 * table lists none) are held at their 18-parameter nominal values. */
static int model9_fixed(int j) { return (j >= 10 && j <= 13) || j >= 15; }

void oracle_tie_model9(float p[NP])
{
    p[1] = p[0]; /* K_SE_ANT = K_SE_AG */
    p[3] = p[2]; /* K_LT_ANT = K_LT_AG */
}

/* Round-0 box: centre = nominal rounded to FP32 (PW from the duration),
 * half-width = frac * centre (0 for parameters a model holds fixed),
 * bounds = centre -/+ half-width in FP32. */
void oracle_initial_box_model(double dur_ms, float frac, int model, float c0[NP], float w0[NP], float lo[NP],
                              float hi[NP])
{
    double nom[NP];
    oracle_nominal(dur_ms, nom);
    for (int j = 0; j < NP; ++j) {
        c0[j] = (float)nom[j];
        w0[j] = (model == 9 && model9_fixed(j)) ? 0.0f : frac * c0[j];
        lo[j] = c0[j] - w0[j];
        hi[j] = c0[j] + w0[j];
    }
}

void oracle_initial_box(double dur_ms, float frac, float c0[NP], float w0[NP], float lo[NP], float hi[NP])
{
    oracle_initial_box_model(dur_ms, frac, 18, c0, w0, lo, hi);
}

/* ------------------------------------------------------------------------- */
/* Scoring many candidates against one saccade (optionally threaded)          */
/* ------------------------------------------------------------------------- */

typedef struct {
    const float* opc; int64_t n0, n1;
    const float* pos; int T, C; double amp, dir, dt; int nsub;
    double* rmse; double* mae;
} score_job;

static void* score_worker(void* arg)
{
    score_job* jb = (score_job*)arg;
    double* th = (double*)malloc(sizeof(double) * (jb->T > 0 ? jb->T : 1));
    for (int64_t i = jb->n0; i < jb->n1; ++i) {
        double p[NP];
        for (int j = 0; j < NP; ++j) p[j] = (double)jb->opc[i * NP + j];
        oracle_simulate(p, jb->amp, jb->T, jb->dt, jb->nsub, th);
        oracle_cost(th, jb->pos, jb->T, jb->C, jb->dir, &jb->rmse[i], jb->mae ? &jb->mae[i] : NULL);
    }
    free(th);
    return NULL;
}

int oracle_score(const float* opc, int64_t n, const float* pos, int T, int C, double amp,
                 double dir_deg, double dt_ms, int nsub, int nthreads, double* rmse, double* mae)
{
    if (n < 0 || T < 1 || (C != 1 && C != 2)) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t tid[256];
    score_job jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (score_job){opc, n * t / nthreads, n * (t + 1) / nthreads, pos, T, C, amp, dir_deg, dt_ms, nsub, rmse, mae};
        if (nthreads > 1) pthread_create(&tid[t], NULL, score_worker, &jobs[t]);
        else score_worker(&jobs[t]);
    }
    if (nthreads > 1)
        for (int t = 0; t < nthreads; ++t) pthread_join(tid[t], NULL);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Box search: candidates, argmin, halving                                    */
/* ------------------------------------------------------------------------- */

/* Fit one saccade.  Round r draws n_cand candidates around centre c^r with
 * half-width w^r (candidate 0 = c^r), scores them all, takes the argmin (lowest
 * RMSE, ties to the lowest index, NaN ranks last), and sets c^{r+1} to the
 * winner and w^{r+1} = shrink * w^r.  c_init (nullable) replaces the nominal
 * round-0 centre (it is clamped into the box; a NaN component keeps the
 * nominal value); w_init_frac scales the round-0
 * half-width relative to the box half-width.  Outputs: the final OPC, its
 * RMSE and mean-abs, and per round the winner index, its RMSE and the centre
 * the round was drawn around (centres: [n_rounds][18], nullable). */
int oracle_fit(const float* pos, int T, int C, double amp, double dir_deg, double dur_ms,
               double dt_ms, uint64_t seed, int64_t n_cand, int n_rounds, float box_frac,
               float w_init_frac, float shrink, const float* c_init, int model, int nsub, int nthreads,
               float opc_out[NP], double* rmse_out, double* mae_out,
               int64_t* best_idx, double* best_rmse, float* centres)
{
    if (n_cand < 1 || n_rounds < 1 || T < 1 || n_cand > 0xFFFFFFFFLL) return -1;
    if (model != 18 && model != 9) return -1;
    float c[NP], w[NP], lo[NP], hi[NP];
    oracle_initial_box_model(dur_ms, box_frac, model, c, w, lo, hi);
    for (int j = 0; j < NP; ++j) w[j] = w[j] * w_init_frac;
    if (c_init)
        for (int j = 0; j < NP; ++j) {
            float v = c_init[(model == 9 && (j == 1 || j == 3)) ? j - 1 : j];
            if (v != v) continue;  /* an unusable (NaN) seed component keeps the nominal centre */
            c[j] = v < lo[j] ? lo[j] : (v > hi[j] ? hi[j] : v);
        }
    float* cand = (float*)malloc(sizeof(float) * NP * n_cand);
    double* cost = (double*)malloc(sizeof(double) * n_cand);
    for (int r = 0; r < n_rounds; ++r) {
        if (centres) memcpy(centres + (size_t)r * NP, c, sizeof c);
        for (int64_t i = 0; i < n_cand; ++i) {
            oracle_candidate(seed, (uint32_t)r, (uint32_t)i, c, w, lo, hi, cand + i * NP);
            if (model == 9) oracle_tie_model9(cand + i * NP);
        }
        oracle_score(cand, n_cand, pos, T, C, amp, dir_deg, dt_ms, nsub, nthreads, cost, NULL);
        int64_t b = 0;
        for (int64_t i = 1; i < n_cand; ++i)
            if (cost[i] < cost[b]) b = i;
        if (best_idx) best_idx[r] = b;
        if (best_rmse) best_rmse[r] = cost[b];
        memcpy(c, cand + b * NP, sizeof c);
        for (int j = 0; j < NP; ++j) w[j] = w[j] * shrink;
    }
    double p[NP];
    for (int j = 0; j < NP; ++j) p[j] = c[j];
    double* th = (double*)malloc(sizeof(double) * T);
    oracle_simulate(p, amp, T, dt_ms, nsub, th);
    oracle_cost(th, pos, T, C, dir_deg, rmse_out, mae_out);
    memcpy(opc_out, c, sizeof c);
    free(th);
    free(cand);
    free(cost);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Nelder-Mead (Section 3.3, Algorithm 1)                                     */
/* ------------------------------------------------------------------------- */

/* The paper's estimator: Nelder-Mead in the variant of Lagarias, Reeds, Wright
 * and Wright (SIAM J. Optim. 9, 1998) -- reflection 1, expansion 2,
 * contraction 1/2, shrink 1/2 -- iterated until the simplex is within TolX of
 * its best vertex in every coordinate AND its values within TolFun of the best
 * value, or until max_iter iterations (Section 3.3).  Coordinates are the OPC
 * relative to nominal (x_j = p_j / nominal_j; the method is affine-equivariant,
 * so this only fixes the units of TolX); the initial simplex is x0 and x0 with
 * one coordinate scaled by 1.05.  The cost is evaluated at the point clamped
 * to [lo_frac, hi_frac] x nominal and rounded to FP32 (the candidate format).
 * Ties in the ordering keep the earlier vertex first (stable insertion). */

typedef struct {
    const float* pos; int T, C; double amp, dir, dt; int nsub;
    double nom[NP]; double lo, hi;
    int64_t nfev;
} nm_problem;

static double nm_cost(nm_problem* pb, const double x[NP])
{
    double p[NP];
    for (int j = 0; j < NP; ++j) {
        double v = x[j];
        if (v < pb->lo) v = pb->lo;
        if (v > pb->hi) v = pb->hi;
        p[j] = (double)(float)(v * pb->nom[j]);
    }
    double* th = (double*)malloc(sizeof(double) * pb->T);
    oracle_simulate(p, pb->amp, pb->T, pb->dt, pb->nsub, th);
    double r, m;
    oracle_cost(th, pb->pos, pb->T, pb->C, pb->dir, &r, &m);
    free(th);
    pb->nfev++;
    return r;
}

/* sort vertices by value, stable: v[(NP+1)][NP], f[NP+1] */
static void nm_sort(double v[][NP], double f[])
{
    for (int i = 1; i <= NP; ++i) {
        double fi = f[i], vi[NP];
        memcpy(vi, v[i], sizeof vi);
        int k = i - 1;
        while (k >= 0 && f[k] > fi) {
            f[k + 1] = f[k];
            memcpy(v[k + 1], v[k], sizeof vi);
            --k;
        }
        f[k + 1] = fi;
        memcpy(v[k + 1], vi, sizeof vi);
    }
}

/* Decision codes: 0 reflect, 1 expand, 2 outside contraction, 3 inside
 * contraction, 4 shrink. */

/* Returns the number of iterations; opc_out gets the best vertex (as FP32 OPC),
 * *f_out its cost.  forced (nullable, [max_iter]): follow these decisions
 * instead of the oracle's own (replay of another implementation's run);
 * own (nullable, [max_iter]) gets the oracle's own decision at every iteration
 * and margin (nullable, [max_iter]) the smallest gap between two values that
 * decision compared. */
int oracle_nelder_mead(const float* pos, int T, int C, double amp, double dir_deg, double dur_ms, double dt_ms,
                       const float* x0_opc, int max_iter, double tol_x, double tol_f, double lo_frac,
                       double hi_frac, int nsub, const signed char* forced, signed char* own, double* margin,
                       float opc_out[NP], double* f_out)
{
    nm_problem pb = {pos, T, C, amp, dir_deg, dt_ms, nsub, {0}, lo_frac, hi_frac, 0};
    oracle_nominal(dur_ms, pb.nom);
    double v[NP + 1][NP], f[NP + 1];
    for (int j = 0; j < NP; ++j) v[0][j] = x0_opc ? (double)x0_opc[j] / pb.nom[j] : 1.0;
    for (int i = 1; i <= NP; ++i) {
        memcpy(v[i], v[0], sizeof v[0]);
        v[i][i - 1] = v[0][i - 1] * 1.05;
    }
    for (int i = 0; i <= NP; ++i) f[i] = nm_cost(&pb, v[i]);
    nm_sort(v, f);
    int it = 0;
    for (; it < max_iter; ++it) {
        double dx = 0.0, df = 0.0;
        for (int i = 1; i <= NP; ++i) {
            df = fmax(df, fabs(f[i] - f[0]));
            for (int j = 0; j < NP; ++j) dx = fmax(dx, fabs(v[i][j] - v[0][j]));
        }
        if (dx <= tol_x && df <= tol_f) break;
        double xb[NP], pt[4][NP], fp[4];
        int have[4] = {0, 0, 0, 0};
        for (int j = 0; j < NP; ++j) {
            double s = 0.0;
            for (int i = 0; i < NP; ++i) s += v[i][j];
            xb[j] = s / NP;
        }
        for (int j = 0; j < NP; ++j) {
            pt[0][j] = xb[j] + (xb[j] - v[NP][j]);         /* reflection          */
            pt[1][j] = xb[j] + 2.0 * (xb[j] - v[NP][j]);   /* expansion           */
            pt[2][j] = xb[j] + 0.5 * (xb[j] - v[NP][j]);   /* outside contraction */
            pt[3][j] = xb[j] - 0.5 * (xb[j] - v[NP][j]);   /* inside contraction  */
        }
#define NM_F(k) (have[k] ? fp[k] : (have[k] = 1, fp[k] = nm_cost(&pb, pt[k])))
        /* the oracle's own decision and the smallest gap it rested on */
        double m = HUGE_VAL;
        int d;
        double fr = NM_F(0);
        m = fmin(m, fabs(fr - f[0]));
        if (fr < f[0]) {
            double fe = NM_F(1);
            m = fmin(m, fabs(fe - fr));
            d = fe < fr ? 1 : 0;
        } else {
            m = fmin(m, fabs(fr - f[NP - 1]));
            if (fr < f[NP - 1]) d = 0;
            else {
                m = fmin(m, fabs(fr - f[NP]));
                if (fr < f[NP]) {
                    double fc = NM_F(2);
                    m = fmin(m, fabs(fc - fr));
                    d = fc <= fr ? 2 : 4;
                } else {
                    double fcc = NM_F(3);
                    m = fmin(m, fabs(fcc - f[NP]));
                    d = fcc < f[NP] ? 3 : 4;
                }
            }
        }
        if (own) own[it] = (signed char)d;
        if (margin) margin[it] = m;
        if (forced) d = forced[it];
        if (d < 4) {
            memcpy(v[NP], pt[d], sizeof pt[d]);
            f[NP] = NM_F(d);
        } else {
            for (int i = 1; i <= NP; ++i) {
                for (int j = 0; j < NP; ++j) v[i][j] = v[0][j] + 0.5 * (v[i][j] - v[0][j]);
                f[i] = nm_cost(&pb, v[i]);
            }
        }
#undef NM_F
        nm_sort(v, f);
    }
    for (int j = 0; j < NP; ++j) {
        double x = v[0][j];
        if (x < lo_frac) x = lo_frac;
        if (x > hi_frac) x = hi_frac;
        opc_out[j] = (float)(x * pb.nom[j]);
    }
    *f_out = f[0];
    return it;
}

/* ------------------------------------------------------------------------- */
/* Gradient-based polish (Section 5: gradient methods as future work)         */
/* ------------------------------------------------------------------------- */

/* Sensitivities d theta_k / d p_j of the RK4 trajectory by central
 * differences with step h_rel * |p_j| (p in double, not rounded).  theta
 * (nullable) [T]; jac [T][NP]. */
int oracle_jacobian(const double p[NP], double amp, int T, double dt_ms, int nsub, double h_rel,
                    double* theta, double* jac)
{
    if (T < 1 || !(h_rel > 0)) return -1;
    double* tp = (double*)malloc(sizeof(double) * T);
    double* tm = (double*)malloc(sizeof(double) * T);
    if (theta) oracle_simulate(p, amp, T, dt_ms, nsub, theta);
    for (int j = 0; j < NP; ++j) {
        double q[NP];
        memcpy(q, p, sizeof q);
        double h = h_rel * fabs(p[j]);
        if (!(h > 0)) h = h_rel;
        q[j] = p[j] + h;
        double hp = q[j] - p[j];
        oracle_simulate(q, amp, T, dt_ms, nsub, tp);
        q[j] = p[j] - h;
        double hm = p[j] - q[j];
        oracle_simulate(q, amp, T, dt_ms, nsub, tm);
        for (int k = 0; k < T; ++k) jac[(int64_t)k * NP + j] = (tp[k] - tm[k]) / (hp + hm);
    }
    free(tp);
    free(tm);
    return 0;
}

/* Solve (H + lam diag H) delta = -g over the n unknowns not held (held
 * unknowns get delta = 0) by a Cholesky factorisation.  H row-major n x n.
 * Returns 0, or -1 if the damped matrix is not positive definite. */
int oracle_damped_solve(int n, const double* H, const double* g, double lam, const int* held, double* delta)
{
    double A[NP][NP], L[NP][NP], y[NP];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (held[i] || held[j]) A[i][j] = (i == j) ? 1.0 : 0.0;
            else A[i][j] = H[i * n + j] + ((i == j) ? lam * H[i * n + j] : 0.0);
        }
    for (int j = 0; j < n; ++j) {
        double d = A[j][j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (!(d > 0)) return -1;
        L[j][j] = sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double s = A[i][j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            L[i][j] = s / L[j][j];
        }
    }
    for (int i = 0; i < n; ++i) { /* L y = -g */
        double s = held[i] ? 0.0 : -g[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) { /* L^T delta = y */
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= L[k][i] * delta[k];
        delta[i] = s / L[i][i];
    }
    return 0;
}

typedef struct {
    const float* pos; int T, C; double amp, u[2], dt; int nsub, objective;
    double nom[NP];
} lm_problem;

/* objective at the FP32-rounded OPC of relative point x: sum of squared or of
 * absolute differences over all samples and channels */
static double lm_cost(const lm_problem* pb, const double x[NP], double* sq_out, double* ab_out)
{
    double p[NP];
    for (int j = 0; j < NP; ++j) p[j] = (double)(float)(x[j] * pb->nom[j]);
    double* th = (double*)malloc(sizeof(double) * pb->T);
    oracle_simulate(p, pb->amp, pb->T, pb->dt, pb->nsub, th);
    double sq = 0.0, ab = 0.0;
    for (int k = 0; k < pb->T; ++k)
        for (int c = 0; c < pb->C; ++c) {
            double e = th[k] * pb->u[c] - (double)pb->pos[k * pb->C + c];
            sq += e * e;
            ab += fabs(e);
        }
    free(th);
    if (sq_out) *sq_out = sq;
    if (ab_out) *ab_out = ab;
    double f = pb->objective == 1 ? ab : sq;
    return (f >= 0.0 && f <= HUGE_VAL && f == f) ? f : HUGE_VAL;
}

/* Levenberg-Marquardt with Marquardt scaling on the relative coordinates
 * x_j = p_j / nominal_j.  Per iteration:
 *   1. residuals e (per sample and channel) of the FP32-rounded point and
 *      their Jacobian J with respect to the free coordinates;
 *   2. weights: 1 for the squared objective; 1/max(|e|, 1e-3) for the
 *      absolute objective (iteratively reweighted least squares);
 *      H = J^T W J, g = J^T W e;
 *   3. a free coordinate is held if H_jj <= 0 or it sits at a bound with
 *      the gradient pointing out of the box;
 *   4. for each factor m of {1e-4, ..., 1e3}: delta_m solves
 *      (H + lam*fac_m diag H) delta = -g, trial point clamp(x + delta_m);
 *   5. the trial with the smallest objective (first on ties) is taken if it
 *      is below the current objective: lam <- lam * fac_best / 10; else
 *      lam <- lam * 1e8 and x stays;
 *   6. stop when a taken step gained <= tol_f times the new objective, when
 *      lam > 1e30, or after max_iter iterations.
 * model 9: free coordinates K_SE (both muscles), K_LT (both), B_AG, B_ANT,
 * B_P, N_C_AG, N_C_ANT, J and N_C_FIX; the rest keep their input values.
 * forced (nullable, [max_iter]): take these decisions (index or -1) for
 * exactly max_iter iterations instead; own/margin (nullable, [max_iter]) get
 * the oracle's own decision and the smallest gap it rested on; fhist
 * (nullable, [max_iter]) the objective at the start of each iteration.
 * Returns the number of iterations; opc_out the result (FP32), *f_out its
 * objective. */
int oracle_polish(const float* pos, int T, int C, double amp, double dir_deg, double dur_ms, double dt_ms,
                  const float* x0_opc, int model, int objective, int max_iter, double tol_f, double lam0,
                  double box_frac, int nsub, double h_rel, const signed char* forced, signed char* own,
                  double* margin, double* fhist, float opc_out[NP], double* f_out)
{
    static const double fac[8] = {1e-4, 1e-3, 1e-2, 1e-1, 1.0, 1e1, 1e2, 1e3};
    lm_problem pb;
    pb.pos = pos; pb.T = T; pb.C = C; pb.amp = amp; pb.dt = dt_ms; pb.nsub = nsub; pb.objective = objective;
    double phi = dir_deg * (M_PI / 180.0);
    pb.u[0] = cos(phi);
    pb.u[1] = sin(phi);
    if (C == 1) { pb.u[0] = dir_deg == 0.0 ? 1.0 : -1.0; pb.u[1] = 0.0; }
    oracle_nominal(dur_ms, pb.nom);

    /* free coordinates and the second component each one moves (ties) */
    int fr[NP], tie[NP], nf = 0;
    for (int j = 0; j < NP; ++j) {
        if (model == 9 && (model9_fixed(j) || j == 1 || j == 3)) continue;
        fr[nf] = j;
        tie[nf] = (model == 9 && (j == 0 || j == 2)) ? j + 1 : -1;
        ++nf;
    }
    double x[NP], lo[NP], hi[NP];
    for (int j = 0; j < NP; ++j) x[j] = (double)x0_opc[j] / pb.nom[j];
    if (model == 9) { /* the antagonist's K_SE and K_LT take the agonist's values */
        x[1] = (double)(float)(x[0] * pb.nom[0]) / pb.nom[1];
        x[3] = (double)(float)(x[2] * pb.nom[2]) / pb.nom[3];
    }
    for (int j = 0; j < NP; ++j) {
        int fixed = model == 9 && model9_fixed(j);
        lo[j] = fixed ? x[j] : 1.0 - box_frac;
        hi[j] = fixed ? x[j] : 1.0 + box_frac;
        if (x[j] < lo[j]) x[j] = lo[j];
        if (x[j] > hi[j]) x[j] = hi[j];
    }
    const int nch = T * C;
    double* th = (double*)malloc(sizeof(double) * T);
    double* ja = (double*)malloc(sizeof(double) * T * NP);
    double* jr = (double*)malloc(sizeof(double) * T * NP);
    double lam = lam0;
    int it = 0;
    for (; it < max_iter; ++it) {
        /* 1-2: normal equations at x */
        double p[NP];
        for (int j = 0; j < NP; ++j) p[j] = (double)(float)(x[j] * pb.nom[j]);
        oracle_jacobian(p, amp, T, dt_ms, nsub, h_rel, th, ja);
        for (int k = 0; k < T; ++k)
            for (int f = 0; f < nf; ++f) {
                double v = pb.nom[fr[f]] * ja[(int64_t)k * NP + fr[f]];
                if (tie[f] >= 0) v += pb.nom[tie[f]] * ja[(int64_t)k * NP + tie[f]];
                jr[(int64_t)k * NP + f] = v;
            }
        double H[NP * NP], g[NP], fcur = 0.0;
        memset(H, 0, sizeof H);
        memset(g, 0, sizeof g);
        for (int k = 0; k < T; ++k)
            for (int c = 0; c < C; ++c) {
                double e = th[k] * pb.u[c] - (double)pos[k * C + c];
                double w = objective == 1 ? 1.0 / fmax(fabs(e), 1e-3) : 1.0;
                fcur += objective == 1 ? fabs(e) : e * e;
                for (int a = 0; a < nf; ++a) {
                    double ja_ = jr[(int64_t)k * NP + a] * pb.u[c];
                    g[a] += w * ja_ * e;
                    for (int b = 0; b < nf; ++b) H[a * nf + b] += w * ja_ * jr[(int64_t)k * NP + b] * pb.u[c];
                }
            }
        (void)nch;
        if (fhist) fhist[it] = fcur;
        /* 3 */
        int held[NP];
        for (int f = 0; f < nf; ++f) {
            int j = fr[f];
            held[f] = !(H[f * nf + f] > 0.0) || (x[j] <= lo[j] && g[f] > 0.0) || (x[j] >= hi[j] && g[f] < 0.0);
        }
        /* 4 */
        double xt[8][NP], ft[8];
        for (int m = 0; m < 8; ++m) {
            double delta[NP];
            memcpy(xt[m], x, sizeof x);
            if (oracle_damped_solve(nf, H, g, lam * fac[m], held, delta) != 0) { ft[m] = HUGE_VAL; continue; }
            for (int f = 0; f < nf; ++f) {
                int j = fr[f];
                double v = x[j] + delta[f];
                if (v < lo[j]) v = lo[j];
                if (v > hi[j]) v = hi[j];
                xt[m][j] = v;
                if (tie[f] >= 0) xt[m][tie[f]] = v;
            }
            ft[m] = lm_cost(&pb, xt[m], NULL, NULL);
        }
        /* 5 */
        int best = 0;
        for (int m = 1; m < 8; ++m)
            if (ft[m] < ft[best]) best = m;
        int d = ft[best] < fcur ? best : -1;
        double mg = fabs(ft[best] - fcur);
        for (int m = 0; m < 8; ++m)
            if (m != best && ft[m] < HUGE_VAL) mg = fmin(mg, fabs(ft[m] - ft[best]));
        if (own) own[it] = (signed char)d;
        if (margin) margin[it] = mg;
        if (forced) d = forced[it];
        int done;
        if (d >= 0) {
            double gain = fcur - ft[d];
            memcpy(x, xt[d], sizeof x);
            lam = lam * fac[d] * 0.1;
            done = gain <= tol_f * ft[d];
        } else {
            lam *= 1e8;
            done = !(lam <= 1e30);
        }
        if (!forced && done) { ++it; break; }
    }
    for (int j = 0; j < NP; ++j) opc_out[j] = (float)(x[j] * pb.nom[j]);
    double sq;
    *f_out = lm_cost(&pb, x, &sq, NULL);
    free(th);
    free(ja);
    free(jr);
    return it;
}
