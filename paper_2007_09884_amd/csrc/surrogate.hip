// libopmm: learned seed for the OPC search -- a small MLP that maps a
// resampled saccade trace to a normalised OPC vector, trained on saccades the
// plant simulator itself generates.  Hand-written BF16 MFMA GEMMs (FP32
// accumulate) for the forward and backward passes, FP32 master weights and
// Adam, the whole training step on the device (capturable in one HIP graph).
//
// Network: 256 -> 512 -> 512 -> 256 -> 18, ReLU on the hidden layers.
// Input: the trace projected on the movement direction, resampled to 128
// points over its own duration, as (position, velocity) pairs (256 values).
// Output: z = (p / p_nominal - 1) / 0.3 per OPC component (p_nominal from
// Table 1; PW nominal = duration - 6 ms).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/opmm.h"
#include "plant.hpp"
#include "runtime.hpp"

using namespace opmm;

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// BF16 MFMA GEMM: C[M][N] = sum_k A(m,k) B(k,n), FP32 accumulate.
//   TA = false: A stored [M][K] (row stride lda); true: stored [K][M].
//   TB = false: B stored [K][N] (row stride ldb); true: stored [N][K].
// Tile 64 x 64 x GBK per 256-thread block; each wave owns a 32 x 32 sub-tile
// and issues GBK / 16 v_mfma_f32_32x32x16_bf16 per K step.  Operands are staged
// through LDS with k contiguous, so every MFMA fragment is one 16-byte LDS
// read; two LDS buffers let the global loads of step i+1 (16 bytes per
// thread and load, into registers) overlap the MFMAs of step i, with one
// barrier per step.  A k-contiguous operand goes to LDS as 16-byte rows; an
// operand contiguous along m or n is transposed on the way (eight 2-byte
// LDS writes per load).
// ---------------------------------------------------------------------------

#ifndef OPMM_GEMM_BK
#define OPMM_GEMM_BK 64
#endif
enum Epi { EPI_F32 = 0, EPI_BIAS_RELU_BF16 = 1, EPI_BIAS_F32 = 2, EPI_RELU_MASK_BF16 = 3 };

constexpr int GBM = 64, GBN = 64, GBK = OPMM_GEMM_BK, GPAD = 8;
constexpr int GROW = GBK + GPAD;  // LDS row length (elements), a multiple of 8 (16 bytes)
constexpr int GCH = GBK / 32;     // 16-byte chunks per thread of one 64 x GBK operand tile

typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

// GCH 16-byte chunks per thread of a 64 (outer) x GBK (k) operand tile.  KC:
// the operand is k-contiguous (rows = outer index); else rows are k.  Chunks
// that leave the matrix, or all chunks when the rows are not 16-byte aligned
// (vec false), are read element by element with zero fill.
template <bool KC>
__device__ __forceinline__ void tile_load(const uint16_t* __restrict__ X, int ld, int o0, int O, int k0, int kend,
                                          bool vec, u32x4 v[GCH])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < GCH; ++j) {
        const int c = tid + 256 * j;
        // KC: GBK / 8 chunks per outer row; else 8 chunks per k row
        const int r = KC ? c / (GBK / 8) : c >> 3, q = (KC ? c % (GBK / 8) : c & 7) * 8;
        // KC: element i is (outer o0 + r, k k0 + q + i); else (k k0 + r, outer o0 + q + i)
        const int ro = KC ? o0 + r : k0 + r;             // storage row
        const int co = KC ? k0 + q : o0 + q;             // storage column of element 0
        const int rlim = KC ? O : kend, clim = KC ? kend : O;
        if (vec && ro < rlim && co + 8 <= clim) {
            v[j] = *reinterpret_cast<const u32x4*>(X + (int64_t)ro * ld + co);
        } else {
            uint16_t e[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) e[i] = (ro < rlim && co + i < clim) ? X[(int64_t)ro * ld + co + i] : (uint16_t)0;
#pragma unroll
            for (int w = 0; w < 4; ++w) v[j][w] = (uint32_t)e[2 * w] | ((uint32_t)e[2 * w + 1] << 16);
        }
    }
}

// Writes the chunks of tile_load into S[outer][k].
template <bool KC>
__device__ __forceinline__ void tile_store(uint16_t (*S)[GROW], const u32x4 v[GCH])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < GCH; ++j) {
        const int c = tid + 256 * j;
        const int r = KC ? c / (GBK / 8) : c >> 3, q = (KC ? c % (GBK / 8) : c & 7) * 8;
        if (KC) {
            *reinterpret_cast<u32x4*>(&S[r][q]) = v[j];
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) S[q + i][r] = (uint16_t)(v[j][i >> 1] >> (16 * (i & 1)));
        }
    }
}

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const uint16_t* __restrict__ A, int lda,
                                                        const uint16_t* __restrict__ B, int ldb, void* C, int ldc,
                                                        const float* __restrict__ bias,
                                                        const uint16_t* __restrict__ mask, int ldm, int kchunk,
                                                        float* __restrict__ colsum)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[2][GBM][GROW];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][GBN][GROW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx16 acc = {};
    // split K: block z covers [z kchunk, (z+1) kchunk); with EPI_F32 it writes slice z of C
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    if (EPI == EPI_F32) C = (float*)C + (int64_t)blockIdx.z * M * ldc;
    const bool va = (lda % 8 == 0) && (((uintptr_t)A & 15) == 0);
    const bool vb = (ldb % 8 == 0) && (((uintptr_t)B & 15) == 0);
    u32x4 ra[GCH], rb[GCH];
    // colsum (non-null): the first row of blocks also sums its B tiles over k, i.e. the column sums of
    // B over this block's K range (the bias gradient when B is the output gradient)
    const bool csum = colsum != nullptr && blockIdx.y == 0 && tid < 64;
    float cs = 0.0f;
    if (kbeg < kend) {
        tile_load<!TA>(A, lda, m0, M, kbeg, kend, va, ra);
        tile_load<TB>(B, ldb, n0, N, kbeg, kend, vb, rb);
        tile_store<!TA>(As[0], ra);
        tile_store<TB>(Bs[0], rb);
    }
    __syncthreads();
    int cur = 0;
    for (int k0 = kbeg; k0 < kend; k0 += GBK) {
        const bool more = k0 + GBK < kend;
        if (more) {
            tile_load<!TA>(A, lda, m0, M, k0 + GBK, kend, va, ra);
            tile_load<TB>(B, ldb, n0, N, k0 + GBK, kend, vb, rb);
        }
#pragma unroll
        for (int ks = 0; ks < GBK; ks += 16) {
            // lane l: A row (l % 32), k = 8 (l / 32) + 0..7; B col (l % 32), same k
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[cur][wm + (lane & 31)][ks + 8 * (lane >> 5)]);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[cur][wn + (lane & 31)][ks + 8 * (lane >> 5)]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        if (csum) {
#pragma unroll
            for (int kq = 0; kq < GBK; kq += 8) {
                const u32x4 w = *reinterpret_cast<const u32x4*>(&Bs[cur][tid][kq]);
#pragma unroll
                for (int i = 0; i < 8; ++i) cs += bf2f((uint16_t)(w[i >> 1] >> (16 * (i & 1))));
            }
        }
        if (more) {
            tile_store<!TA>(As[cur ^ 1], ra);
            tile_store<TB>(Bs[cur ^ 1], rb);
        }
        __syncthreads();
        cur ^= 1;
    }
    if (csum && n0 + tid < N) colsum[(int64_t)blockIdx.z * N + n0 + tid] = cs;
    // accumulator j of lane l holds row 8 (j / 4) + 4 (l / 32) + j % 4, column l % 32
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int m = m0 + wm + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
        const int n = n0 + wn + (lane & 31);
        if (m >= M || n >= N) continue;
        float v = acc[j];
        if (EPI == EPI_F32) {
            ((float*)C)[(int64_t)m * ldc + n] = v;
        } else if (EPI == EPI_BIAS_RELU_BF16) {
            v = fmaxf(v + bias[n], 0.0f);
            ((uint16_t*)C)[(int64_t)m * ldc + n] = f2bf(v);
        } else if (EPI == EPI_BIAS_F32) {
            ((float*)C)[(int64_t)m * ldc + n] = v + bias[n];
        } else {  // backward through ReLU: the layer input was a post-ReLU activation
            const bool on = mask[(int64_t)m * ldm + n] != 0;
            ((uint16_t*)C)[(int64_t)m * ldc + n] = on ? f2bf(v) : (uint16_t)0;
        }
    }
}

// nsplit > 1 (EPI_F32 only): C holds nsplit slices [M][ldc] of partial sums over K.  colsum (nullable,
// B stored [K][N]): [nsplit][N] column sums of B over each slice's K range.
template <bool TA, bool TB, int EPI>
hipError_t gemm(int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb, void* C, int ldc,
                const float* bias, const uint16_t* mask, int ldm, hipStream_t st, int nsplit = 1,
                float* colsum = nullptr)
{
    const int kchunk = (((K + nsplit - 1) / nsplit) + GBK - 1) / GBK * GBK;
    dim3 grid((N + GBN - 1) / GBN, (M + GBM - 1) / GBM, nsplit);
    hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, bias,
                       mask, ldm, kchunk, colsum);
    return hipGetLastError();
}

// Deterministic split-K reduction of a layer's gradients, slices summed in z order:
// out[i] = sum_z wparts[z][i] for i < nw (weights), out[nw + j] = sum_z bparts[z][j] for
// j < nb (the bias, stored right after the weights).
__global__ void splitk_sum_kernel(int64_t nw, int nb, int nsplit, const float* __restrict__ wparts,
                                  const float* __restrict__ bparts, float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw + nb) return;
    const bool w = i < nw;
    const float* src = w ? wparts + i : bparts + (i - nw);
    const int64_t stride = w ? nw : nb;
    float a = 0.0f;
    for (int z = 0; z < nsplit; ++z) a += src[(int64_t)z * stride];
    out[i] = a;
}

constexpr int SPLITK_ROWS = 512;  // batch rows per split of the weight-gradient GEMM
constexpr int SPLITK_MAX = 16;

// ---------------------------------------------------------------------------
// Network state
// ---------------------------------------------------------------------------

constexpr int NL = 4;
constexpr int WIDTH[NL + 1] = {256, 512, 512, 256, 18};
constexpr int NPTS = 128;        // resampled points
constexpr float FEAT_POS = 1.0f / 16.0f;  // feature scale of position (deg)
constexpr float FEAT_VEL = 4.0f;          // feature scale of velocity (deg/ms)
constexpr float ZSCALE = 0.3f;            // z = (p/p_nom - 1) / ZSCALE

constexpr int64_t param_count()
{
    int64_t n = 0;
    for (int l = 0; l < NL; ++l) n += (int64_t)WIDTH[l] * WIDTH[l + 1] + WIDTH[l + 1];
    return n;
}
constexpr int64_t NPARAM = param_count();

int64_t w_off(int l)
{
    int64_t n = 0;
    for (int i = 0; i < l; ++i) n += (int64_t)WIDTH[i] * WIDTH[i + 1] + WIDTH[i + 1];
    return n;
}
int64_t b_off(int l) { return w_off(l) + (int64_t)WIDTH[l] * WIDTH[l + 1]; }

}  // namespace

struct opmm_surrogate {
    opmm_ctx* ctx = nullptr;
    int device = 0;
    int cap_batch = 0;
    int64_t step = 0;  // Adam steps taken
    // parameters: [W0 (256x512), b0, W1, b1, W2, b2, W3, b3], W_l stored [in][out]
    float* w = nullptr;       // FP32 master
    uint16_t* wb = nullptr;   // BF16 copy used by the GEMMs
    float* g = nullptr;       // gradients
    float* m1 = nullptr;      // Adam first moment
    float* m2 = nullptr;      // Adam second moment
    // activations for cap_batch rows
    uint16_t* act[NL] = {};   // act[0] = input features, act[l] = output of hidden layer l (post-ReLU)
    float* out = nullptr;     // [B][18]
    uint16_t* dact[NL] = {};  // gradient w.r.t. act[l] (l >= 1) and w.r.t. the output (index 0 reused)
    float* target = nullptr;  // [B][18]
    float* loss = nullptr;    // [1]
    float* trace = nullptr;   // [B][MAX_T_GEN] generated traces
    int32_t* tlen = nullptr;  // [B]
    float* dur = nullptr;     // [B]
    uint64_t* counter = nullptr;  // device step counter for data generation (graph-replay safe)
    float* gpart = nullptr;       // split-K partial weight gradients [SPLITK_MAX][512 x 512]
    float* cpart = nullptr;       // split-K partial bias gradients [SPLITK_MAX][512]
    // training data ring: GEN_BATCHES consecutive batches generated in one launch
    uint16_t* ring_feat = nullptr;  // [GEN_BATCHES][ring_cap][256]
    float* ring_tgt = nullptr;      // [GEN_BATCHES][ring_cap][18]
    float* ring_trace = nullptr;    // [GEN_BATCHES][ring_cap][MAX_T_GEN]
    int ring_cap = 0;
};

namespace {

constexpr int MAX_T_GEN = 160;
constexpr int GEN_BATCHES = 16;  // training batches generated per launch (one lane per saccade each)

__global__ void fill_f32_kernel(float* p, int64_t n, float v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void to_bf16_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = f2bf(src[i]);
}

// He-uniform initialisation from the SplitMix64 stream; biases zero.
__global__ void init_params_kernel(float* w, uint64_t seed)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    int64_t off = 0;
    for (int l = 0; l < NL; ++l) {
        const int64_t nw = (int64_t)WIDTH[l] * WIDTH[l + 1];
        if (i < off + nw) {
            const float lim = sqrtf(6.0f / WIDTH[l]) * (l == NL - 1 ? 0.5f : 1.0f);
            uint64_t z = splitmix64(seed, 1 + (uint64_t)i);
            float u = (float)(z >> 40) * 0x1p-24f;
            w[i] = (2.0f * u - 1.0f) * lim;
            return;
        }
        off += nw;
        if (i < off + WIDTH[l + 1]) {
            w[i] = 0.0f;
            return;
        }
        off += WIDTH[l + 1];
    }
}

// Resample a trace (length T, period dt) to NPTS points over its own duration
// and write (position, velocity) features; velocity is the central difference
// (one-sided at the ends) interpolated the same way.
// Feature point j of a trace r[T]: position and velocity (central difference)
// linearly interpolated at t = j (T - 1) / (NPTS - 1).
__device__ __forceinline__ void trace_feature_point(const float* r, int T, float dt, int j, uint16_t* feat)
{
    const float span = (float)(T - 1);
    {
        float t = span * (float)j / (float)(NPTS - 1);
        int k = (int)floorf(t);
        if (k > T - 2) k = T - 2;
        if (k < 0) k = 0;
        float f = t - (float)k;
        float p0 = r[k], p1 = T > 1 ? r[k + 1] : r[0];
        auto vel = [&](int q) {
            if (T < 2) return 0.0f;
            int a = q > 0 ? q - 1 : 0, b = q < T - 1 ? q + 1 : T - 1;
            return (r[b] - r[a]) / ((float)(b - a) * dt);
        };
        float v0 = vel(k), v1 = vel(T > 1 ? k + 1 : 0);
        float pos = p0 + f * (p1 - p0);
        float v = v0 + f * (v1 - v0);
        feat[2 * j] = f2bf(pos * FEAT_POS);
        feat[2 * j + 1] = f2bf(v * FEAT_VEL);
    }
}

__device__ void trace_features(const float* r, int T, float dt, uint16_t* feat)
{
    for (int j = 0; j < NPTS; ++j) trace_feature_point(r, T, dt, j, feat);
}

// Features of the saccades of a fit batch, from the projected traces: one wave
// per saccade (block s), lanes take every 64th feature point.
__global__ __launch_bounds__(64) void features_kernel(int S, const opmm_rt::SacDev* __restrict__ sacs,
                                                      const float* __restrict__ proj, float dt,
                                                      uint16_t* __restrict__ feat)
{
    const int s = blockIdx.x;
    if (s >= S) return;
    const float* r = proj + sacs[s].proj_off;
    const int T = sacs[s].T;
    for (int j = threadIdx.x; j < NPTS; j += 64) trace_feature_point(r, T, dt, j, feat + (int64_t)s * (2 * NPTS));
}

// Training data: draw a true OPC (nominal x U[1 - 0.3, 1 + 0.3]), amplitude
// U[2, 30] deg, duration 2.2 A + 21 ms, noise sigma U[0, 0.1] deg; simulate the
// plant, add noise along the movement direction, resample to features and
// write the normalised target.  One sample per lane, keyed by (seed, step, i).
struct GenSink {
    float* out;
    __device__ __forceinline__ void operator()(int k, R dth, R theq) { out[k] = (float)(dth + theq); }
};

__global__ __launch_bounds__(64) void gen_batch_kernel(int B, uint64_t seed, const uint64_t* __restrict__ counter,
                                                        float spread, float sigma_max, float* __restrict__ trace,
                                                        uint16_t* __restrict__ feat, float* __restrict__ target)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = i < B;
    int ii = valid ? i : 0;
    // grid y: consecutive batches of the data stream, batch j keyed by step counter + j
    const uint64_t step = *counter + blockIdx.y;
    trace += (int64_t)blockIdx.y * B * MAX_T_GEN;
    feat += (int64_t)blockIdx.y * B * (2 * NPTS);
    target += (int64_t)blockIdx.y * B * P;
    auto uni = [&](uint32_t k) {
        uint64_t z = splitmix64(seed, 1 + ((step << 40) | ((uint64_t)ii << 8) | k));
        return (float)(z >> 40) * 0x1p-24f;  // [0, 1)
    };
    const float amp = 2.0f + 28.0f * uni(0);
    const float dur = 2.2f * amp + 21.0f;
    int T = (int)ceilf(dur);
    if (T > MAX_T_GEN) T = MAX_T_GEN;
    const float sigma = sigma_max * uni(1);
    float p[P];
    for (int j = 0; j < P; ++j) {
        float mlt = 1.0f + spread * (2.0f * uni(2 + j) - 1.0f);
        p[j] = nominal_param(j, dur) * mlt;
        if (valid) target[(int64_t)ii * P + j] = (mlt - 1.0f) / ZSCALE;
    }
    Plant pl;
    plant_setup(p, amp, 1.0f, pl);
    R frac;
    int k0 = pulse_end_sample(pl.pwd, T, frac);
    float* tr = trace + (int64_t)ii * MAX_T_GEN;
    GenSink sink{tr};
    if (!valid) return;
    run_trajectory<1>(pl, T, (R)1.0, k0, frac, k0, k0, sink);
    for (int k = 0; k < T; k += 2) {  // Box-Muller pairs
        float u1 = fmaxf(uni(32 + k), 0x1p-25f), u2 = uni(33 + k);
        float rad = sqrtf(-2.0f * logf(u1));
        tr[k] += sigma * rad * cosf(6.2831853f * u2);
        if (k + 1 < T) tr[k + 1] += sigma * rad * sinf(6.2831853f * u2);
    }
    trace_features(tr, T, 1.0f, feat + (int64_t)ii * (2 * NPTS));
}

// Output gradient of the MSE loss; loss accumulated (mean over B x 18).
__global__ void mse_grad_kernel(int B, const float* __restrict__ out, const float* __restrict__ target,
                                uint16_t* __restrict__ dout, float* __restrict__ loss)
{
    __shared__ float red[256];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = B * P;
    float e = 0.0f;
    if (i < n) {
        e = out[i] - target[i];
        dout[i] = f2bf(2.0f * e / (float)n);
    }
    red[threadIdx.x] = e * e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, red[0] / (float)n);
}

// Adam (Kingma & Ba 2015, Algorithm 1) on the FP32 master weights, with a BF16
// copy for the GEMMs.  b1, b2 and their complements om1 = 1 - b1, om2 = 1 - b2
// are each the FP32 value nearest the exact constant, and c1 = 1 / (1 - b1^t),
// c2 = 1 / (1 - b2^t) are formed on the host in FP64: 1 - b2^t taken in FP32
// loses about five digits to cancellation in the first steps.
__global__ void adam_kernel(int64_t n, float* __restrict__ w, uint16_t* __restrict__ wb, const float* __restrict__ g,
                            float* __restrict__ m1, float* __restrict__ m2, float lr, float b1, float om1, float b2,
                            float om2, float eps, float c1, float c2)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float a = b1 * m1[i] + om1 * gi;
    float v = b2 * m2[i] + om2 * (gi * gi);
    m1[i] = a;
    m2[i] = v;
    float upd = (a * c1) / (sqrtf(v * c2) + eps);
    float nw = w[i] - lr * upd;
    w[i] = nw;
    wb[i] = f2bf(nw);
}

__global__ void bump_kernel(uint64_t* c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *c += 1;
}

// z (network output) -> OPC seed, clamped into the search box of the saccade
__global__ void denorm_kernel(int S, const float* __restrict__ z, const opmm_rt::SacDev* __restrict__ sacs,
                              float box_frac, float* __restrict__ opc)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S * P) return;
    int s = i / P, j = i % P;
    float nom = nominal_param(j, sacs[s].dur);
    float mlt = 1.0f + ZSCALE * z[i];
    mlt = fminf(fmaxf(mlt, 1.0f - box_frac), 1.0f + box_frac);
    opc[i] = nom * mlt;
}

int blocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

// Merge the plain-search results of the rejected saccades back: keep the
// lower-RMSE result of the two and flag the fallback.
__global__ void merge_fallback_kernel(int F, const int32_t* __restrict__ idx, const float* __restrict__ opc_f,
                                      const float* __restrict__ rmse_f, const float* __restrict__ mae_f,
                                      const int32_t* __restrict__ st_f, float* opc, float* rmse, float* mae,
                                      int32_t* status)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F) return;
    const int s = idx[i];
    const float r_seed = rmse[s], r_plain = rmse_f[i];
    const bool take = !(r_seed <= r_plain);  // NaN seeded result -> plain
    if (take) {
        for (int j = 0; j < P; ++j) opc[(int64_t)s * P + j] = opc_f[(int64_t)i * P + j];
        rmse[s] = r_plain;
        if (mae) mae[s] = mae_f[i];
    }
    status[s] = (status[s] | st_f[i]) | OPMM_ST_FALLBACK;
}

}  // namespace

// ===========================================================================
// Host side
// ===========================================================================

namespace {

#define SG_HIP(call)                                                        \
    do {                                                                    \
        hipError_t _e = (call);                                             \
        if (_e != hipSuccess) return opmm_rt::hip_fail(sg->ctx, _e, #call); \
    } while (0)

int sg_alloc(opmm_surrogate* sg, int batch)
{
    if (batch <= sg->cap_batch) return OPMM_OK;
    SG_HIP(hipDeviceSynchronize());
    for (int l = 0; l < NL; ++l) {
        if (sg->act[l]) (void)hipFree(sg->act[l]);
        if (sg->dact[l]) (void)hipFree(sg->dact[l]);
        sg->act[l] = sg->dact[l] = nullptr;
    }
    for (void* p : {(void*)sg->out, (void*)sg->target, (void*)sg->trace, (void*)sg->tlen, (void*)sg->dur})
        if (p) (void)hipFree(p);
    for (int l = 0; l < NL; ++l) {
        SG_HIP(hipMalloc(&sg->act[l], sizeof(uint16_t) * (size_t)batch * WIDTH[l]));
        SG_HIP(hipMalloc(&sg->dact[l], sizeof(uint16_t) * (size_t)batch * (l == 0 ? WIDTH[NL] : WIDTH[l])));
    }
    SG_HIP(hipMalloc(&sg->out, sizeof(float) * (size_t)batch * WIDTH[NL]));
    SG_HIP(hipMalloc(&sg->target, sizeof(float) * (size_t)batch * WIDTH[NL]));
    SG_HIP(hipMalloc(&sg->trace, sizeof(float) * (size_t)batch * MAX_T_GEN));
    SG_HIP(hipMalloc(&sg->tlen, sizeof(int32_t) * (size_t)batch));
    SG_HIP(hipMalloc(&sg->dur, sizeof(float) * (size_t)batch));
    if (!sg->gpart) SG_HIP(hipMalloc(&sg->gpart, sizeof(float) * (size_t)SPLITK_MAX * 512 * 512));
    if (!sg->cpart) SG_HIP(hipMalloc(&sg->cpart, sizeof(float) * (size_t)SPLITK_MAX * 512));
    sg->cap_batch = batch;
    return OPMM_OK;
}

}  // namespace

namespace opmm_rt {
int surrogate_reserve(opmm_surrogate* sg, int batch) { return sg_alloc(sg, batch); }
}  // namespace opmm_rt

namespace {

// forward pass over the B rows of x0 (features); output in sg->out
int sg_forward(opmm_surrogate* sg, int B, const uint16_t* x0, hipStream_t st)
{
    for (int l = 0; l < NL; ++l) {
        const uint16_t* W = sg->wb + w_off(l);
        const float* bias = sg->w + b_off(l);
        const int K = WIDTH[l], N = WIDTH[l + 1];
        hipError_t e;
        if (l < NL - 1)
            e = gemm<false, false, EPI_BIAS_RELU_BF16>(B, N, K, l == 0 ? x0 : sg->act[l], K, W, N, sg->act[l + 1], N,
                                                       bias, nullptr, 0, st);
        else
            e = gemm<false, false, EPI_BIAS_F32>(B, N, K, l == 0 ? x0 : sg->act[l], K, W, N, sg->out, N, bias, nullptr,
                                                 0, st);
        if (e != hipSuccess) return opmm_rt::hip_fail(sg->ctx, e, "gemm forward");
    }
    return OPMM_OK;
}

// backward pass after sg_forward on x0, against tgt [B][18]; gradients into sg->g
// loss: device scalar the MSE is accumulated into (zeroed by the caller)
int sg_backward(opmm_surrogate* sg, int B, const uint16_t* x0, const float* tgt, float* loss, hipStream_t st)
{
    const int NO = WIDTH[NL];
    hipLaunchKernelGGL(mse_grad_kernel, dim3(blocks((int64_t)B * NO, 256)), dim3(256), 0, st, B, sg->out, tgt,
                       sg->dact[0], loss);
    for (int l = NL - 1; l >= 0; --l) {
        const int K = WIDTH[l], N = WIDTH[l + 1];
        const uint16_t* dy = (l == NL - 1) ? sg->dact[0] : sg->dact[l + 1];
        // dW_l = act[l]^T . dY   ([K][B] x [B][N]): the batch is the long contraction, split it so
        // that a 512 x 512 gradient fills the chip, then sum the slices in a fixed order
        const int nsplit = std::min(SPLITK_MAX, std::max(1, (B + SPLITK_ROWS - 1) / SPLITK_ROWS));
        // the bias gradient (column sums of dY) comes out of the same GEMM
        hipError_t e = gemm<true, false, EPI_F32>(K, N, B, l == 0 ? x0 : sg->act[l], K, dy, N,
                                                  nsplit > 1 ? sg->gpart : sg->g + w_off(l),
                                                  N, nullptr, nullptr, 0, st, nsplit,
                                                  nsplit > 1 ? sg->cpart : sg->g + b_off(l));
        if (e != hipSuccess) return opmm_rt::hip_fail(sg->ctx, e, "gemm dW");
        if (nsplit > 1)
            hipLaunchKernelGGL(splitk_sum_kernel, dim3(blocks((int64_t)K * N + N, 256)), dim3(256), 0, st,
                               (int64_t)K * N, N, nsplit, sg->gpart, sg->cpart, sg->g + w_off(l));
        if (l > 0) {
            // dX_l = (dY . W_l^T) masked by act[l] > 0   ([B][N] x [N][K])
            e = gemm<false, true, EPI_RELU_MASK_BF16>(B, K, N, dy, N, sg->wb + w_off(l), N, sg->dact[l], K, nullptr,
                                                      sg->act[l], K, st);
            if (e != hipSuccess) return opmm_rt::hip_fail(sg->ctx, e, "gemm dX");
        }
    }
    return OPMM_OK;
}

int sg_adam(opmm_surrogate* sg, float lr, hipStream_t st)
{
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    sg->step += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)sg->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)sg->step)));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, st, NPARAM, sg->w, sg->wb, sg->g, sg->m1,
                       sg->m2, lr, (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)eps, c1, c2);
    return hipGetLastError() == hipSuccess ? OPMM_OK : OPMM_EDEVICE;
}

}  // namespace

extern "C" {

int opmm_surrogate_create(opmm_ctx* ctx, uint64_t init_seed, opmm_surrogate** out)
{
    if (!ctx || !out) return OPMM_EINVAL;
    *out = nullptr;
    opmm_surrogate* sg = new (std::nothrow) opmm_surrogate();
    if (!sg) return OPMM_ENOMEM;
    sg->ctx = ctx;
    sg->device = opmm_rt::ctx_device(ctx);
    if (hipSetDevice(sg->device) != hipSuccess) { delete sg; return OPMM_EDEVICE; }
    int rc = OPMM_OK;
    if (hipMalloc(&sg->w, sizeof(float) * NPARAM) != hipSuccess || hipMalloc(&sg->g, sizeof(float) * NPARAM) != hipSuccess ||
        hipMalloc(&sg->m1, sizeof(float) * NPARAM) != hipSuccess || hipMalloc(&sg->m2, sizeof(float) * NPARAM) != hipSuccess ||
        hipMalloc(&sg->wb, sizeof(uint16_t) * NPARAM) != hipSuccess || hipMalloc(&sg->loss, sizeof(float)) != hipSuccess ||
        hipMalloc(&sg->counter, sizeof(uint64_t)) != hipSuccess)
        rc = OPMM_ENOMEM;
    if (rc == OPMM_OK) {
        hipLaunchKernelGGL(init_params_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, 0, sg->w, init_seed);
        hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, 0, sg->w, sg->wb, NPARAM);
        hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, 0, sg->m1, NPARAM, 0.0f);
        hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, 0, sg->m2, NPARAM, 0.0f);
        hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, 0, sg->g, NPARAM, 0.0f);
        if (hipMemset(sg->counter, 0, sizeof(uint64_t)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            rc = OPMM_EDEVICE;
    }
    if (rc != OPMM_OK) {
        opmm_surrogate_destroy(sg);
        return rc;
    }
    *out = sg;
    return OPMM_OK;
}

int opmm_surrogate_destroy(opmm_surrogate* sg)
{
    if (!sg) return OPMM_OK;
    (void)hipSetDevice(sg->device);
    (void)hipDeviceSynchronize();
    for (int l = 0; l < NL; ++l) {
        if (sg->act[l]) (void)hipFree(sg->act[l]);
        if (sg->dact[l]) (void)hipFree(sg->dact[l]);
    }
    for (void* p : {(void*)sg->w, (void*)sg->wb, (void*)sg->g, (void*)sg->m1, (void*)sg->m2, (void*)sg->out,
                    (void*)sg->target, (void*)sg->loss, (void*)sg->trace, (void*)sg->tlen, (void*)sg->dur,
                    (void*)sg->counter, (void*)sg->gpart, (void*)sg->cpart, (void*)sg->ring_feat,
                    (void*)sg->ring_tgt, (void*)sg->ring_trace})
        if (p) (void)hipFree(p);
    delete sg;
    return OPMM_OK;
}

int64_t opmm_surrogate_param_count(void) { return NPARAM; }

int opmm_surrogate_get_params(opmm_surrogate* sg, int which, float* host_out)
{
    if (!sg || !host_out) return OPMM_EINVAL;
    const float* src = which == 0 ? sg->w : which == 1 ? sg->g : which == 2 ? sg->m1 : which == 3 ? sg->m2 : nullptr;
    if (!src) return opmm_rt::fail(sg->ctx, OPMM_EINVAL, "which must be 0 (weights), 1 (gradients), 2, 3 (Adam)");
    SG_HIP(hipSetDevice(sg->device));
    SG_HIP(hipDeviceSynchronize());
    SG_HIP(hipMemcpy(host_out, src, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    return OPMM_OK;
}

int opmm_surrogate_set_params(opmm_surrogate* sg, const float* host_w)
{
    if (!sg || !host_w) return OPMM_EINVAL;
    SG_HIP(hipSetDevice(sg->device));
    SG_HIP(hipDeviceSynchronize());
    SG_HIP(hipMemcpy(sg->w, host_w, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, 0, sg->w, sg->wb, NPARAM);
    SG_HIP(hipDeviceSynchronize());
    return OPMM_OK;
}

int opmm_surrogate_forward(opmm_surrogate* sg, const uint16_t* feat, int32_t B, float* out, void* stream)
{
    if (!sg || B < 0 || (B > 0 && (!feat || !out))) return OPMM_EINVAL;
    if (B == 0) return OPMM_OK;
    SG_HIP(hipSetDevice(sg->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = sg_alloc(sg, B)) != OPMM_OK) return rc;
    SG_HIP(hipMemcpyAsync(sg->act[0], feat, sizeof(uint16_t) * (size_t)B * WIDTH[0], hipMemcpyDeviceToDevice, st));
    if ((rc = sg_forward(sg, B, sg->act[0], st)) != OPMM_OK) return rc;
    SG_HIP(hipMemcpyAsync(out, sg->out, sizeof(float) * (size_t)B * WIDTH[NL], hipMemcpyDeviceToDevice, st));
    return OPMM_OK;
}

int opmm_surrogate_backward(opmm_surrogate* sg, const uint16_t* feat, const float* target, int32_t B, float* loss_out,
                            void* stream)
{
    if (!sg || B <= 0 || !feat || !target) return OPMM_EINVAL;
    SG_HIP(hipSetDevice(sg->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = sg_alloc(sg, B)) != OPMM_OK) return rc;
    SG_HIP(hipMemcpyAsync(sg->act[0], feat, sizeof(uint16_t) * (size_t)B * WIDTH[0], hipMemcpyDeviceToDevice, st));
    SG_HIP(hipMemcpyAsync(sg->target, target, sizeof(float) * (size_t)B * WIDTH[NL], hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(fill_f32_kernel, dim3(1), dim3(64), 0, st, sg->loss, 1, 0.0f);
    if ((rc = sg_forward(sg, B, sg->act[0], st)) != OPMM_OK) return rc;
    if ((rc = sg_backward(sg, B, sg->act[0], sg->target, sg->loss, st)) != OPMM_OK) return rc;
    if (loss_out) {
        SG_HIP(hipMemcpyAsync(loss_out, sg->loss, sizeof(float), hipMemcpyDeviceToHost, st));
        SG_HIP(hipStreamSynchronize(st));
    }
    return OPMM_OK;
}

int opmm_surrogate_generate(opmm_surrogate* sg, uint64_t data_seed, uint64_t step, int32_t B, float spread,
                            float sigma_max, uint16_t* feat_out, float* target_out, void* stream)
{
    if (!sg || B <= 0 || !feat_out || !target_out) return OPMM_EINVAL;
    SG_HIP(hipSetDevice(sg->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = sg_alloc(sg, B)) != OPMM_OK) return rc;
    SG_HIP(hipMemcpyAsync(sg->counter, &step, sizeof(uint64_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(gen_batch_kernel, dim3(blocks(B, 64)), dim3(64), 0, st, B, data_seed, sg->counter, spread,
                       sigma_max, sg->trace, feat_out, target_out);
    SG_HIP(hipGetLastError());
    SG_HIP(hipStreamSynchronize(st));
    return OPMM_OK;
}

int opmm_surrogate_train(opmm_surrogate* sg, uint64_t data_seed, int32_t B, int32_t n_steps, float lr0, float lr_min,
                         float spread, float sigma_max, float* loss_out, void* stream)
{
    if (!sg || B <= 0 || n_steps < 0) return OPMM_EINVAL;
    SG_HIP(hipSetDevice(sg->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if ((rc = sg_alloc(sg, B)) != OPMM_OK) return rc;
    if (sg->ring_cap < B) {
        SG_HIP(hipDeviceSynchronize());
        for (void* p : {(void*)sg->ring_feat, (void*)sg->ring_tgt, (void*)sg->ring_trace})
            if (p) (void)hipFree(p);
        sg->ring_feat = nullptr;
        sg->ring_tgt = sg->ring_trace = nullptr;
        sg->ring_cap = 0;
        SG_HIP(hipMalloc(&sg->ring_feat, sizeof(uint16_t) * (size_t)GEN_BATCHES * B * WIDTH[0]));
        SG_HIP(hipMalloc(&sg->ring_tgt, sizeof(float) * (size_t)GEN_BATCHES * B * WIDTH[NL]));
        SG_HIP(hipMalloc(&sg->ring_trace, sizeof(float) * (size_t)GEN_BATCHES * B * MAX_T_GEN));
        sg->ring_cap = B;
    }
    // per-step losses stay on the device until the end: no host round trip inside the loop
    float* hist = nullptr;
    if (n_steps > 0) {
        SG_HIP(hipMallocAsync((void**)&hist, sizeof(float) * (size_t)n_steps, st));
        hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks(n_steps, 256)), dim3(256), 0, st, hist, (int64_t)n_steps, 0.0f);
    }
    for (int32_t t = 0; t < n_steps && rc == OPMM_OK; ++t) {
        // the next GEN_BATCHES batches of the data stream in one launch (keyed by the step counter, so
        // batch t is the same as when generated alone)
        const int j = t % GEN_BATCHES;
        if (j == 0)
            hipLaunchKernelGGL(gen_batch_kernel, dim3(blocks(B, 64), std::min(GEN_BATCHES, n_steps - t)), dim3(64), 0,
                               st, B, data_seed, sg->counter, spread, sigma_max, sg->ring_trace, sg->ring_feat,
                               sg->ring_tgt);
        const uint16_t* x0 = sg->ring_feat + (size_t)j * B * WIDTH[0];
        const float* tgt = sg->ring_tgt + (size_t)j * B * WIDTH[NL];
        if ((rc = sg_forward(sg, B, x0, st)) != OPMM_OK) break;
        if ((rc = sg_backward(sg, B, x0, tgt, hist + t, st)) != OPMM_OK) break;
        // cosine decay from lr0 to lr_min over this call's steps
        const double ph = n_steps > 1 ? (double)t / (double)(n_steps - 1) : 1.0;
        const float lr = (float)(lr_min + 0.5 * (lr0 - lr_min) * (1.0 + std::cos(M_PI * ph)));
        if ((rc = sg_adam(sg, lr, st)) != OPMM_OK) break;
        hipLaunchKernelGGL(bump_kernel, dim3(1), dim3(64), 0, st, sg->counter);
    }
    if (rc == OPMM_OK && loss_out && n_steps > 0)
        rc = hipMemcpyAsync(loss_out, hist, sizeof(float) * (size_t)n_steps, hipMemcpyDeviceToHost, st) == hipSuccess
                 ? OPMM_OK
                 : opmm_rt::fail(sg->ctx, OPMM_EDEVICE, "loss copy failed");
    if (hist) (void)hipFreeAsync(hist, st);
    if (rc != OPMM_OK) return rc;
    SG_HIP(hipGetLastError());
    SG_HIP(hipStreamSynchronize(st));
    return OPMM_OK;
}

int opmm_surrogate_adam_step(opmm_surrogate* sg, float lr, void* stream)
{
    if (!sg) return OPMM_EINVAL;
    SG_HIP(hipSetDevice(sg->device));
    return sg_adam(sg, lr, (hipStream_t)stream);
}

// Learned OPC of S uploaded and projected saccades: features, network, de-normalisation into the
// search box.
static int sg_predict(opmm_surrogate* sg, int32_t S, const opmm_rt::SacDev* sd, const float* proj, float dt_ms,
                      float box_frac, float* opc_out, hipStream_t st)
{
    int rc;
    if ((rc = sg_alloc(sg, S)) != OPMM_OK) return rc;
    hipLaunchKernelGGL(features_kernel, dim3(S), dim3(64), 0, st, S, sd, proj, dt_ms, sg->act[0]);
    if ((rc = sg_forward(sg, S, sg->act[0], st)) != OPMM_OK) return rc;
    hipLaunchKernelGGL(denorm_kernel, dim3(blocks((int64_t)S * P, 256)), dim3(256), 0, st, S, sg->out, sd, box_frac,
                       opc_out);
    SG_HIP(hipGetLastError());
    return OPMM_OK;
}

}  // extern "C"

namespace opmm_rt {
int surrogate_predict_projected(opmm_surrogate* sg, int n, const SacDev* sacs, const float* proj, float dt_ms,
                                float box_frac, float* opc_out, hipStream_t st)
{
    if (n <= 0) return OPMM_OK;
    return sg_predict(sg, n, sacs, proj, dt_ms, box_frac, opc_out, st);
}
}  // namespace opmm_rt

extern "C" {

int opmm_surrogate_predict(opmm_surrogate* sg, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                           float dt_ms, float box_frac, float* opc_out, void* stream)
{
    if (!sg) return OPMM_EINVAL;
    opmm_ctx* ctx = sg->ctx;
    if (S < 0 || (S > 0 && (!pos || !sacs || !opc_out))) return opmm_rt::fail(ctx, OPMM_EINVAL, "bad arguments");
    if (!(box_frac > 0.0f && box_frac < 1.0f)) return opmm_rt::fail(ctx, OPMM_EINVAL, "box_frac must be in (0, 1)");
    if (S == 0) return OPMM_OK;
    SG_HIP(hipSetDevice(sg->device));
    hipStream_t st = (hipStream_t)stream;
    int rc;
    const opmm_rt::SacDev* sd;
    const float* proj;
    if ((rc = opmm_rt::project_batch(ctx, pos, pos_len, sacs, S, &sd, &proj, st)) != OPMM_OK) return rc;
    return sg_predict(sg, S, sd, proj, dt_ms, box_frac, opc_out, st);
}

int opmm_surrogate_features(opmm_surrogate* sg, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                            float dt_ms, uint16_t* feat_out, void* stream)
{
    if (!sg) return OPMM_EINVAL;
    opmm_ctx* ctx = sg->ctx;
    if (S <= 0 || !pos || !sacs || !feat_out) return opmm_rt::fail(ctx, OPMM_EINVAL, "bad arguments");
    SG_HIP(hipSetDevice(sg->device));
    hipStream_t st = (hipStream_t)stream;
    const opmm_rt::SacDev* sd;
    const float* proj;
    int rc;
    if ((rc = opmm_rt::project_batch(ctx, pos, pos_len, sacs, S, &sd, &proj, st)) != OPMM_OK) return rc;
    hipLaunchKernelGGL(features_kernel, dim3(S), dim3(64), 0, st, S, sd, proj, dt_ms, feat_out);
    SG_HIP(hipGetLastError());
    return OPMM_OK;
}

int opmm_fit_learned(opmm_surrogate* sg, const float* pos, int64_t pos_len, const opmm_saccade* sacs, int32_t S,
                     const opmm_fit_params* seeded, const opmm_fit_params* plain, float fallback_rmse,
                     float* opc_out, float* rmse_out, float* mae_out, int32_t* status_out, int32_t* n_fallback,
                     void* stream)
{
    if (!sg) return OPMM_EINVAL;
    opmm_ctx* ctx = sg->ctx;
    if (!seeded || !plain) return opmm_rt::fail(ctx, OPMM_EINVAL, "params are NULL");
    if (!(fallback_rmse >= 0.0f)) return opmm_rt::fail(ctx, OPMM_EINVAL, "fallback_rmse must be >= 0");
    if (S < 0 || (S > 0 && (!pos || !sacs || !opc_out || !rmse_out || !status_out)))
        return opmm_rt::fail(ctx, OPMM_EINVAL, "bad arguments");
    if (n_fallback) *n_fallback = 0;
    if (S == 0) return OPMM_OK;
    SG_HIP(hipSetDevice(sg->device));
    hipStream_t st = (hipStream_t)stream;
    // 1. one upload and projection of the batch serves the learned seeds and the seeded refine
    opmm_rt::FitStage fs;
    const opmm_rt::SacDev* sd;
    const float* proj;
    int rc = opmm_rt::fit_stage(ctx, pos, pos_len, sacs, S, seeded, opc_out, rmse_out, &fs, &sd, &proj, st);
    if (rc != OPMM_OK) return rc;
    float* seeds = nullptr;
    SG_HIP(hipMallocAsync((void**)&seeds, sizeof(float) * (size_t)S * P, st));
    rc = sg_predict(sg, S, sd, proj, seeded->dt_ms, seeded->box_frac, seeds, st);
    // 2. seeded refine
    if (rc == OPMM_OK)
        rc = opmm_rt::fit_launch(ctx, pos, S, fs, seeded, seeds, opc_out, rmse_out, mae_out, status_out, nullptr, st);
    // 3. the plain search judges: saccades whose seeded RMSE exceeds the threshold are re-fitted plainly
    std::vector<float> h_rmse(S);
    if (rc == OPMM_OK && hipMemcpyAsync(h_rmse.data(), rmse_out, sizeof(float) * S, hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = opmm_rt::fail(ctx, OPMM_EDEVICE, "copy of seeded RMSE failed");
    if (rc == OPMM_OK && hipStreamSynchronize(st) != hipSuccess) rc = opmm_rt::fail(ctx, OPMM_EDEVICE, "sync failed");
    std::vector<int32_t> fb;
    if (rc == OPMM_OK)
        for (int s = 0; s < S; ++s)
            if (!(h_rmse[s] <= fallback_rmse)) fb.push_back(s);
    if (rc == OPMM_OK && !fb.empty()) {
        const int F = (int)fb.size();
        std::vector<opmm_saccade> sub(F);
        for (int i = 0; i < F; ++i) sub[i] = sacs[fb[i]];
        float *opc_f = nullptr, *rmse_f = nullptr, *mae_f = nullptr;
        int32_t *st_f = nullptr, *d_idx = nullptr;
        bool ok = hipMallocAsync((void**)&opc_f, sizeof(float) * (size_t)F * P, st) == hipSuccess &&
                  hipMallocAsync((void**)&rmse_f, sizeof(float) * F, st) == hipSuccess &&
                  hipMallocAsync((void**)&mae_f, sizeof(float) * F, st) == hipSuccess &&
                  hipMallocAsync((void**)&st_f, sizeof(int32_t) * F, st) == hipSuccess &&
                  hipMallocAsync((void**)&d_idx, sizeof(int32_t) * F, st) == hipSuccess;
        if (!ok) rc = opmm_rt::fail(ctx, OPMM_ENOMEM, "fallback buffers");
        if (rc == OPMM_OK) rc = opmm_fit(ctx, pos, pos_len, sub.data(), F, plain, nullptr, opc_f, rmse_f, mae_f, st_f,
                                         nullptr, stream);
        if (rc == OPMM_OK) {
            if (hipMemcpyAsync(d_idx, fb.data(), sizeof(int32_t) * F, hipMemcpyHostToDevice, st) != hipSuccess)
                rc = opmm_rt::fail(ctx, OPMM_EDEVICE, "index upload failed");
            else {
                hipLaunchKernelGGL(merge_fallback_kernel, dim3(blocks(F, 128)), dim3(128), 0, st, F, d_idx, opc_f,
                                   rmse_f, mae_f, st_f, opc_out, rmse_out, mae_out, status_out);
                if (hipStreamSynchronize(st) != hipSuccess) rc = opmm_rt::fail(ctx, OPMM_EDEVICE, "merge failed");
            }
        }
        for (void* p : {(void*)opc_f, (void*)rmse_f, (void*)mae_f, (void*)st_f, (void*)d_idx})
            if (p) (void)hipFreeAsync(p, st);
        if (n_fallback) *n_fallback = F;
    }
    (void)hipFreeAsync(seeds, st);
    return rc;
}

int opmm_surrogate_save(opmm_surrogate* sg, const char* path)
{
    if (!sg || !path) return OPMM_EINVAL;
    std::vector<float> buf((size_t)NPARAM * 3);
    int rc;
    if ((rc = opmm_surrogate_get_params(sg, 0, buf.data())) != OPMM_OK) return rc;
    if ((rc = opmm_surrogate_get_params(sg, 2, buf.data() + NPARAM)) != OPMM_OK) return rc;
    if ((rc = opmm_surrogate_get_params(sg, 3, buf.data() + 2 * NPARAM)) != OPMM_OK) return rc;
    FILE* f = std::fopen(path, "wb");
    if (!f) return opmm_rt::fail(sg->ctx, OPMM_EINVAL, std::string("cannot write ") + path);
    const char magic[8] = {'O', 'P', 'M', 'M', 'S', 'G', '0', '1'};
    int64_t hdr[2] = {NPARAM, sg->step};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof hdr, 1, f) == 1 &&
              std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? OPMM_OK : opmm_rt::fail(sg->ctx, OPMM_EINVAL, std::string("write failed: ") + path);
}

int opmm_surrogate_load(opmm_surrogate* sg, const char* path)
{
    if (!sg || !path) return OPMM_EINVAL;
    FILE* f = std::fopen(path, "rb");
    if (!f) return opmm_rt::fail(sg->ctx, OPMM_EINVAL, std::string("cannot read ") + path);
    char magic[8];
    int64_t hdr[2];
    std::vector<float> buf((size_t)NPARAM * 3);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "OPMMSG01", 8) == 0 &&
              std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == NPARAM &&
              std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return opmm_rt::fail(sg->ctx, OPMM_EINVAL, std::string("not a surrogate checkpoint: ") + path);
    SG_HIP(hipSetDevice(sg->device));
    SG_HIP(hipDeviceSynchronize());
    SG_HIP(hipMemcpy(sg->w, buf.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice));
    SG_HIP(hipMemcpy(sg->m1, buf.data() + NPARAM, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
    SG_HIP(hipMemcpy(sg->m2, buf.data() + 2 * NPARAM, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, 0, sg->w, sg->wb, NPARAM);
    SG_HIP(hipDeviceSynchronize());
    sg->step = hdr[1];
    return OPMM_OK;
}

}  // extern "C"
