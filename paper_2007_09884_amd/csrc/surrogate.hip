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
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4_t;

// FP32 -> BF16, round to nearest even; a NaN stays a (quiet) NaN.  Branch-free: it runs on every
// element the network writes.
__device__ __forceinline__ uint16_t f2bf(float f)
{
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
    return (uint16_t)((u & 0x7FFFFFFFu) > 0x7F800000u ? ((u >> 16) | 0x40u) : r);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// Network shape and the BF16 weight layouts the MFMA kernels read
// ---------------------------------------------------------------------------

constexpr int NL = 4;
constexpr int WIDTH[NL + 1] = {256, 512, 512, 256, 18};
constexpr int NPAD[NL] = {512, 512, 256, 32};  // layer outputs padded to whole 32-column MFMA tiles

// Each layer's weights exist twice in BF16, padded to NPAD columns with zeros, each in the order
// the MFMA B fragments are read: for output tile t (32 columns) and contraction step s (16
// indices) the 64 lanes' fragments (8 contraction indices of one column each) are 1 KB in a row,
// so a wave's fragment load is one contiguous read.
//   forward  WF_l: output = layer output n, contraction = layer input k;
//   backward WB_l: output = layer input k, contraction = layer output n (the dX pass).
__host__ __device__ constexpr int64_t wpack_off(int l)
{
    int64_t n = 0;
    for (int i = 0; i < l; ++i) n += (int64_t)NPAD[i] * WIDTH[i];
    return n;
}
constexpr int64_t NPACK = wpack_off(NL);

// Position of W_l[k][n] in a fragment-ordered layout with `out` the output index (tile out / 32,
// lane column out % 32) and `in` the contraction index (step in / 16, lane half (in % 16) / 8,
// element in % 8); nsteps = contraction length / 16.
__host__ __device__ __forceinline__ int64_t frag_index(int out, int in, int nsteps)
{
    return ((int64_t)((out >> 5) * nsteps + (in >> 4)) * 64 + (out & 31) + 32 * ((in & 15) >> 3)) * 8 + (in & 7);
}
__host__ __device__ __forceinline__ int64_t wf_index(int l, int k, int n)
{
    return wpack_off(l) + frag_index(n, k, WIDTH[l] / 16);
}
__host__ __device__ __forceinline__ int64_t wb_index(int l, int k, int n)
{
    return wpack_off(l) + frag_index(k, n, NPAD[l] / 16);
}

// ---------------------------------------------------------------------------
// MFMA building blocks: v_mfma_f32_32x32x16_bf16, 64-wide waves.  Fragment
// layout (checked against a CPU matmul): lane l supplies A row (l % 32) and B
// column (l % 32), contraction indices 8 (l / 32) + 0..7; accumulator j of
// lane l is row 8 (j / 4) + 4 (l / 32) + j % 4, column l % 32.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int acc_row(int j, int lane) { return 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3); }

// NT 32-column tiles of a 32-row product  X[32][KC] . Bop, X in LDS (row stride xs elements), Bop a
// fragment-ordered weight layout in global memory (L2-resident).  The B fragments run PF contraction
// steps ahead in registers (a Ring): the global latency hides behind the MFMAs of the steps between.
// A ring is started, i.e. its first PF fragments requested, before the product that uses it, so a
// layer's first loads overlap the previous layer's epilogue and barrier.
#ifndef OPMM_MLP_PF
#define OPMM_MLP_PF 4  // contraction steps of B fragments in flight per product (2, 3, 6, 8, 16: slower)
#endif

template <int KC, int NT>
struct Ring {
    static constexpr int NS = KC / 16;
    static constexpr int PF = NS < OPMM_MLP_PF ? NS : OPMM_MLP_PF;
    const uint16_t* bp[NT];
    bf16x8 q[PF][NT];
    __device__ __forceinline__ void start(const uint16_t* __restrict__ Bg, const int (&n0)[NT])
    {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int t = 0; t < NT; ++t) bp[t] = Bg + ((int64_t)(n0[t] >> 5) * NS * 64 + lane) * 8;
#pragma unroll
        for (int i = 0; i < PF; ++i)
#pragma unroll
            for (int t = 0; t < NT; ++t) q[i][t] = *reinterpret_cast<const bf16x8*>(bp[t] + 512 * i);
        __builtin_amdgcn_sched_barrier(0);
    }
};

template <int KC, int NT>
__device__ __forceinline__ void mma_rows32(const uint16_t* X, int xs, Ring<KC, NT>& r, floatx16 (&acc)[NT])
{
    constexpr int NS = Ring<KC, NT>::NS, PF = Ring<KC, NT>::PF;
    constexpr int PA = NS < 4 ? NS : 4;  // A fragments (LDS) in flight
    const int lane = threadIdx.x & 63;
    const uint16_t* xa = X + (lane & 31) * xs + 8 * (lane >> 5);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = floatx16{};
    bf16x8 aq[PA];
#pragma unroll
    for (int i = 0; i < PA; ++i) aq[i] = *reinterpret_cast<const bf16x8*>(xa + 16 * i);
    // the scheduling barriers keep each refill where it is written: left alone, the scheduler sinks the
    // loads next to their MFMAs and only one or two stay in flight
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ks = 0; ks < NS; ++ks) {
        const bf16x8 a = aq[ks % PA];
        if (ks + PA < NS) aq[ks % PA] = *reinterpret_cast<const bf16x8*>(xa + 16 * (ks + PA));
        bf16x8 b[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            b[t] = r.q[ks % PF][t];
            if (ks + PF < NS) r.q[ks % PF][t] = *reinterpret_cast<const bf16x8*>(r.bp[t] + 512 * (ks + PF));
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[t], acc[t], 0, 0, 0);
    }
}


// ---------------------------------------------------------------------------
// Fused network pass: one block of 8 waves per 32 batch rows, every layer's
// activations in LDS.  Forward: H1..H3 = ReLU(H_l W_l + b_l) in BF16, output
// H3 W3 + b3 in FP32.  TRAIN also takes the loss and back-propagates the
// output gradient through the hidden layers (each gradient overwrites, in
// place, the activation that gives its ReLU mask), and writes to global
// memory what the weight-gradient kernel contracts over the batch: the
// activations H1..H3 and the gradients G0..G3 of each layer's output
// (G3 = dLoss/dOut padded to 32 columns, in BF16).
// ---------------------------------------------------------------------------

constexpr int FR = 32;       // batch rows per block
constexpr int FTHREADS = 512;
constexpr int XPAD = 8;      // LDS row padding (elements): rows shift by 16 bytes across banks

struct MlpSmem {
    uint16_t h0[FR][256 + XPAD];
    uint16_t h1[FR][512 + XPAD];
    uint16_t h2[FR][512 + XPAD];
    uint16_t h3[FR][256 + XPAD];
    uint16_t d3[FR][32 + XPAD];
    float red[FTHREADS / 64];
};

struct MlpArgs {
    int B;
    int Bp;                 // (TRAIN) row stride of the transposed operands: B rounded up to DW_BK
    const uint16_t* x0;     // [B][256]
    const uint16_t* wf;     // forward layouts
    const uint16_t* wbk;    // backward layouts
    const float* w;         // FP32 parameters (biases read from here)
    float* out;             // [B][18] (forward only), nullable in TRAIN
    const float* target;    // [B][18] (TRAIN)
    float* loss;            // (TRAIN) mean squared error added here
    uint16_t* ht[NL];       // (TRAIN) layer inputs H_0 = x0 .. H_3, transposed: [WIDTH[l]][Bp], zero past B
    uint16_t* gt[NL];       // (TRAIN) output gradients G_0 .. G_3, transposed: [NPAD[l]][Bp], zero past B
};

// Lane's four consecutive rows 8q + 4 (lane / 32) + 0..3 of accumulator group q (j = 4q .. 4q + 3) as
// one 8-byte store into a transposed operand T[col][row0 + row] (rows past B written as zeros).
__device__ __forceinline__ void store_t4(uint16_t* __restrict__ T, int64_t ld, int col, int row0, int B, int q,
                                         int lane, const uint16_t (&h)[16])
{
    const int r = row0 + 8 * q + 4 * (lane >> 5);
    uint32_t lo = 0, hi = 0;
    if (r + 0 < B) lo |= (uint32_t)h[4 * q + 0];
    if (r + 1 < B) lo |= (uint32_t)h[4 * q + 1] << 16;
    if (r + 2 < B) hi |= (uint32_t)h[4 * q + 2];
    if (r + 3 < B) hi |= (uint32_t)h[4 * q + 3] << 16;
    *reinterpret_cast<uint2*>(T + (int64_t)col * ld + r) = make_uint2(lo, hi);
}

__host__ __device__ constexpr int64_t w_off_c(int l)
{
    int64_t n = 0;
    for (int i = 0; i < l; ++i) n += (int64_t)WIDTH[i] * WIDTH[i + 1] + WIDTH[i + 1];
    return n;
}
__host__ __device__ constexpr int64_t b_off_c(int l) { return w_off_c(l) + (int64_t)WIDTH[l] * WIDTH[l + 1]; }
constexpr int64_t NPARAM_C = w_off_c(NL);

// Epilogue of a hidden layer's forward product: Y = ReLU(acc + b) in BF16 for the block's 32 rows;
// HT (nullable): also the transposed copy for the weight gradients.
template <int NT>
__device__ __forceinline__ void fwd_epilogue(const floatx16 (&acc)[NT], const int (&n0)[NT], uint16_t* Y, int ys,
                                             const float* bias, uint16_t* HT, int ld, int row0, int B)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = n0[t] + (lane & 31);
        const float bv = bias[col];
        uint16_t h[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            h[j] = f2bf(fmaxf(acc[t][j] + bv, 0.0f));
            Y[acc_row(j, lane) * ys + col] = h[j];
        }
        if (HT)
#pragma unroll
            for (int q = 0; q < 4; ++q) store_t4(HT, ld, col, row0, B, q, lane, h);
    }
}

// Epilogue of a backward product through hidden layer l: G_{l-1} = acc masked by H_l > 0, written over
// H_l (which holds the mask) -- each element is read and written by the same lane -- and transposed
// into GT.
template <int NT>
__device__ __forceinline__ void bwd_epilogue(const floatx16 (&acc)[NT], const int (&n0)[NT], uint16_t* HM, int hs,
                                             uint16_t* GT, int ld, int row0, int B)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = n0[t] + (lane & 31);
        uint16_t gv[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            uint16_t& h = HM[acc_row(j, lane) * hs + col];
            gv[j] = h != 0 ? f2bf(acc[t][j]) : (uint16_t)0;
            h = gv[j];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) store_t4(GT, ld, col, row0, B, q, lane, gv);
    }
}

// Wave w owns output tiles {w, w + 8} of a 512-wide product and tile w of a 256-wide one; wave 0 also
// computes the 32-wide output layer.  Each product's ring is started before the previous epilogue.
template <bool TRAIN>
__global__ __launch_bounds__(FTHREADS) void mlp_pass_kernel(MlpArgs A)
{
    __shared__ __attribute__((aligned(16))) MlpSmem sm;
    const int r0 = blockIdx.x * FR;
    const int nrows = max(0, min(FR, A.B - r0));
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ld = A.Bp;
    const int n512[2] = {32 * wave, 32 * (wave + 8)};
    const int n256[1] = {32 * wave};
    const int n32[1] = {0};
    Ring<256, 2> rf0;
    rf0.start(A.wf + wpack_off(0), n512);
    // stage the input rows (zeros past the batch)
    for (int c = tid; c < FR * 32; c += FTHREADS) {
        const int r = c >> 5, q = (c & 31) * 8;
        u32x4_t v = {0u, 0u, 0u, 0u};
        if (r < nrows) v = *reinterpret_cast<const u32x4_t*>(A.x0 + (int64_t)(r0 + r) * 256 + q);
        *reinterpret_cast<u32x4_t*>(&sm.h0[r][q]) = v;
    }
    __syncthreads();
    if (TRAIN) {  // H_0 transposed: thread c takes feature c % 256, rows 8 (c / 256) .. + 7
        for (int c = tid; c < 256 * 4; c += FTHREADS) {
            const int f = c & 255, rq = (c >> 8) * 8;
            uint32_t v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = (uint32_t)sm.h0[rq + 2 * i][f] | ((uint32_t)sm.h0[rq + 2 * i + 1][f] << 16);
            *reinterpret_cast<u32x4_t*>(A.ht[0] + (int64_t)f * ld + r0 + rq) = u32x4_t{v[0], v[1], v[2], v[3]};
        }
    }
    floatx16 acc2[2], acc1[1];
    // H1 = ReLU(H0 W0 + b0)
    mma_rows32<256, 2>(&sm.h0[0][0], 256 + XPAD, rf0, acc2);
    Ring<512, 2> rf1;
    rf1.start(A.wf + wpack_off(1), n512);
    fwd_epilogue<2>(acc2, n512, &sm.h1[0][0], 512 + XPAD, A.w + b_off_c(0), TRAIN ? A.ht[1] : nullptr, ld, r0, A.B);
    __syncthreads();
    // H2 = ReLU(H1 W1 + b1)
    mma_rows32<512, 2>(&sm.h1[0][0], 512 + XPAD, rf1, acc2);
    Ring<512, 1> rf2;
    rf2.start(A.wf + wpack_off(2), n256);
    fwd_epilogue<2>(acc2, n512, &sm.h2[0][0], 512 + XPAD, A.w + b_off_c(1), TRAIN ? A.ht[2] : nullptr, ld, r0, A.B);
    __syncthreads();
    // H3 = ReLU(H2 W2 + b2)
    mma_rows32<512, 1>(&sm.h2[0][0], 512 + XPAD, rf2, acc1);
    Ring<256, 1> rf3;
    Ring<32, 1> rb3;
    if (wave == 0) rf3.start(A.wf + wpack_off(3), n32);
    else if (TRAIN) rb3.start(A.wbk + wpack_off(3), n256);
    fwd_epilogue<1>(acc1, n256, &sm.h3[0][0], 256 + XPAD, A.w + b_off_c(2), TRAIN ? A.ht[3] : nullptr, ld, r0, A.B);
    __syncthreads();
    // output layer (one 32-column tile, 18 used): wave 0
    if (wave == 0) {
        mma_rows32<256, 1>(&sm.h3[0][0], 256 + XPAD, rf3, acc1);
        if (TRAIN) rb3.start(A.wbk + wpack_off(3), n256);
        const int col = lane & 31;
        const float bv = col < 18 ? A.w[b_off_c(3) + col] : 0.0f;
        const float nf = (float)(A.B * 18);
        float sq = 0.0f;
        uint16_t gv[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int r = acc_row(j, lane);
            const bool ok = r < nrows && col < 18;
            const float o = acc1[0][j] + bv;
            if (!TRAIN) {
                if (ok) A.out[(int64_t)(r0 + r) * 18 + col] = o;
            } else {
                float e = 0.0f;
                if (ok) e = o - A.target[(int64_t)(r0 + r) * 18 + col];
                sq += e * e;
                gv[j] = ok ? f2bf(2.0f * e / nf) : (uint16_t)0;
                sm.d3[r][col] = gv[j];
            }
        }
        if (TRAIN) {
#pragma unroll
            for (int q = 0; q < 4; ++q) store_t4(A.gt[3], ld, col, r0, A.B, q, lane, gv);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) sq += __shfl_xor(sq, o);
            if (lane == 0) atomicAdd(A.loss, sq / nf);
        }
    }
    if (!TRAIN) return;
    __syncthreads();
    // G2 = (G3 W3^T) . [H3 > 0]   (contraction over the 32 padded outputs)
    mma_rows32<32, 1>(&sm.d3[0][0], 32 + XPAD, rb3, acc1);
    Ring<256, 2> rb2;
    rb2.start(A.wbk + wpack_off(2), n512);
    bwd_epilogue<1>(acc1, n256, &sm.h3[0][0], 256 + XPAD, A.gt[2], ld, r0, A.B);
    __syncthreads();
    // G1 = (G2 W2^T) . [H2 > 0]
    mma_rows32<256, 2>(&sm.h3[0][0], 256 + XPAD, rb2, acc2);
    Ring<512, 2> rb1;
    rb1.start(A.wbk + wpack_off(1), n512);
    bwd_epilogue<2>(acc2, n512, &sm.h2[0][0], 512 + XPAD, A.gt[1], ld, r0, A.B);
    __syncthreads();
    // G0 = (G1 W1^T) . [H1 > 0]
    mma_rows32<512, 2>(&sm.h2[0][0], 512 + XPAD, rb1, acc2);
    bwd_epilogue<2>(acc2, n512, &sm.h1[0][0], 512 + XPAD, A.gt[0], ld, r0, A.B);
}

// ---------------------------------------------------------------------------
// Weight gradients of all four layers: dW_l = H_l^T G_l, a contraction over the
// batch, from the transposed operands the pass kernel wrote (batch contiguous,
// zero past B up to Bp).  Split-K: every 64 x 64 output tile runs eight times,
// block 8 t + x contracting tile t over the x-th eighth of the batch into partial
// slice x; grad_reduce_kernel sums the eight slices in a fixed order
// (deterministic) and, when training, takes the Adam step.  A block stages 32
// batch rows per step (20 KB of LDS), so up to eight blocks share a CU: the
// kernel is bound by load latency, and resident blocks are what hides it
// (measured at 4096 rows: 29.5 us with 128-row steps, 2 blocks per CU; 22.5 us
// with 32-row steps; contiguous eighths instead of 32-row segments dealt to the
// slices in turn, 20.8 us).  The first row of tiles also sums its G tiles: the
// bias gradient.
// ---------------------------------------------------------------------------

constexpr int DBM = 64, DBN = 64, DW_BK = 32, DROW = DW_BK + 8;  // batch rows per step (64: slower)
constexpr int DW_CH = DBM * DW_BK / 8 / 256;  // 16-byte chunks per thread and operand tile
constexpr int DW_SLICES = 8;                  // partial gradient slices (split-K over the batch; 4 and 16 were slower)
constexpr int DW_TILES[NL] = {(256 / 64) * (512 / 64), (512 / 64) * (512 / 64), (512 / 64) * (256 / 64),
                              (256 / 64) * 1};
constexpr int DW_BLOCKS = DW_TILES[0] + DW_TILES[1] + DW_TILES[2] + DW_TILES[3];

struct AdamArgs {
    float lr, b1, om1, b2, om2, eps, c1, c2;
};

// Adam (Kingma & Ba 2015, Algorithm 1) on parameter i with gradient gi; weights (wl >= 0: weight of
// layer wl at input row k, output column n) also refresh their two BF16 copies.
__device__ __forceinline__ void adam_update(int64_t i, float gi, float* __restrict__ w, float* __restrict__ m1,
                                            float* __restrict__ m2, const AdamArgs& a, uint16_t* __restrict__ wf,
                                            uint16_t* __restrict__ wbk, int wl, int k, int n)
{
    float mm = a.b1 * m1[i] + a.om1 * gi;
    float vv = a.b2 * m2[i] + a.om2 * (gi * gi);
    m1[i] = mm;
    m2[i] = vv;
    float upd = (mm * a.c1) / (sqrtf(vv * a.c2) + a.eps);
    float nw = w[i] - a.lr * upd;
    w[i] = nw;
    if (wl >= 0) {
        const uint16_t h = f2bf(nw);
        wf[wf_index(wl, k, n)] = h;
        wbk[wb_index(wl, k, n)] = h;
    }
}

// One step of DW_BK = 32 batch columns of a transposed operand X [O][ld] for rows o0 .. o0 + 63 (rows
// >= O read as zeros): batch rows 32 (seg0 + step) .. + 31, zeros from segment seg_end on.  DW_CH
// 16-byte chunks per thread.
__device__ __forceinline__ void dw_load(const uint16_t* __restrict__ X, int64_t ld, int O, int o0, int seg0,
                                        int seg_end, int step, u32x4_t v[DW_CH])
{
#pragma unroll
    for (int j = 0; j < DW_CH; ++j) {
        const int c = threadIdx.x + 256 * j;
        const int r = c / (DW_BK / 8), q = (c % (DW_BK / 8)) * 8;
        const int seg = seg0 + step;
        v[j] = (o0 + r < O && seg < seg_end)
                   ? *reinterpret_cast<const u32x4_t*>(X + (int64_t)(o0 + r) * ld + DW_BK * seg + q)
                   : u32x4_t{0u, 0u, 0u, 0u};
    }
}
__device__ __forceinline__ void dw_store(uint16_t (*S)[DROW], const u32x4_t v[DW_CH])
{
#pragma unroll
    for (int j = 0; j < DW_CH; ++j) {
        const int c = threadIdx.x + 256 * j;
        const int r = c / (DW_BK / 8), q = (c % (DW_BK / 8)) * 8;
        *reinterpret_cast<u32x4_t*>(&S[r][q]) = v[j];
    }
}

struct DwOperands {
    const uint16_t* ht[NL];  // H_l^T [WIDTH[l]][Bp]
    const uint16_t* gt[NL];  // G_l^T [NPAD[l]][Bp]
};

// gpart: DW_SLICES slices of NPARAM partial gradients, slice x over the x-th eighth of the batch rows.
__global__ __launch_bounds__(256) void mlp_dw_kernel(int Bp, DwOperands ops, float* __restrict__ gpart)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[2][DBM][DROW];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][DBN][DROW];
    const int x = blockIdx.x % DW_SLICES;
    // tile -> layer; the largest layer first
    int bid = blockIdx.x / DW_SLICES, l;
    if (bid < DW_TILES[1]) l = 1;
    else if ((bid -= DW_TILES[1]) < DW_TILES[0]) l = 0;
    else if ((bid -= DW_TILES[0]) < DW_TILES[2]) l = 2;
    else { bid -= DW_TILES[2]; l = 3; }
    const int K = WIDTH[l], N = WIDTH[l + 1], NPd = NPAD[l];
    const int ntn = (NPd + DBN - 1) / DBN;
    const int m0 = (bid / ntn) * DBM, n0 = (bid % ntn) * DBN;
    const uint16_t* H = ops.ht[l];
    const uint16_t* G = ops.gt[l];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int nseg_all = Bp / DW_BK;                     // DW_BK-row segments of the batch
    const int per = (nseg_all + DW_SLICES - 1) / DW_SLICES;  // segments per slice
    const int seg0 = x * per, seg_end = min(nseg_all, seg0 + per);
    const int nsteps = max(0, seg_end - seg0);
    floatx16 acc = {};
    const bool csum = m0 == 0 && tid < 64;
    float cs = 0.0f;
    u32x4_t ra[DW_CH], rb[DW_CH];
    if (nsteps > 0) {
        dw_load(H, Bp, K, m0, seg0, seg_end, 0, ra);
        dw_load(G, Bp, NPd, n0, seg0, seg_end, 0, rb);
        dw_store(As[0], ra);
        dw_store(Bs[0], rb);
    }
    __syncthreads();
    int cur = 0;
    for (int st = 0; st < nsteps; ++st) {
        const bool more = st + 1 < nsteps;
        if (more) {
            dw_load(H, Bp, K, m0, seg0, seg_end, st + 1, ra);
            dw_load(G, Bp, NPd, n0, seg0, seg_end, st + 1, rb);
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the MFMAs
#pragma unroll
        for (int ks = 0; ks < DW_BK; ks += 16) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[cur][wm + (lane & 31)][ks + 8 * (lane >> 5)]);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[cur][wn + (lane & 31)][ks + 8 * (lane >> 5)]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        if (csum) {
#pragma unroll
            for (int kq = 0; kq < DW_BK; kq += 8) {
                const u32x4_t v = *reinterpret_cast<const u32x4_t*>(&Bs[cur][tid][kq]);
#pragma unroll
                for (int i = 0; i < 8; ++i) cs += bf2f((uint16_t)(v[i >> 1] >> (16 * (i & 1))));
            }
        }
        if (more) {
            dw_store(As[cur ^ 1], ra);
            dw_store(Bs[cur ^ 1], rb);
        }
        __syncthreads();
        cur ^= 1;
    }
    float* gp = gpart + (int64_t)x * NPARAM_C;
    // weights: element (m, n) of dW_l is parameter w_off(l) + m N + n
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int m = m0 + wm + acc_row(j, lane);
        const int n = n0 + wn + (lane & 31);
        if (m < K && n < N) gp[w_off_c(l) + (int64_t)m * N + n] = acc[j];
    }
    // biases: sums of G_l over the batch rows
    if (csum && n0 + tid < N) gp[b_off_c(l) + n0 + tid] = cs;
}

// g = the sum of the DW_SLICES partial slices, in slice order; ADAM: the Adam step on every parameter and
// one bump of the data-generation counter.
template <bool ADAM>
__global__ void grad_reduce_kernel(const float* __restrict__ gpart, float* __restrict__ g, float* __restrict__ w,
                                   float* __restrict__ m1, float* __restrict__ m2, uint16_t* __restrict__ wf,
                                   uint16_t* __restrict__ wbk, AdamArgs a, uint64_t* __restrict__ step_counter)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ADAM && step_counter && i == 0) *step_counter += 1;
    if (i >= NPARAM_C) return;
    float gi = gpart[i];
#pragma unroll
    for (int x = 1; x < DW_SLICES; ++x) gi += gpart[(int64_t)x * NPARAM_C + i];
    g[i] = gi;
    if (ADAM) {
        int l = 0;
        while (l < NL - 1 && i >= w_off_c(l + 1)) ++l;
        const int64_t off = i - w_off_c(l);
        const int N = WIDTH[l + 1];
        const bool is_w = i < b_off_c(l);
        adam_update(i, gi, w, m1, m2, a, wf, wbk, is_w ? l : -1, is_w ? (int)(off / N) : 0, is_w ? (int)(off % N) : 0);
    }
}

// ---------------------------------------------------------------------------
// Network state
// ---------------------------------------------------------------------------

constexpr int NPTS = 128;        // resampled points
constexpr float FEAT_POS = 1.0f / 16.0f;  // feature scale of position (deg)
constexpr float FEAT_VEL = 4.0f;          // feature scale of velocity (deg/ms)
constexpr float ZSCALE = 0.3f;            // z = (p/p_nom - 1) / ZSCALE

constexpr int64_t NPARAM = NPARAM_C;

}  // namespace

struct opmm_surrogate {
    opmm_ctx* ctx = nullptr;
    int device = 0;
    int cap_batch = 0;
    int64_t step = 0;  // Adam steps taken
    // parameters: [W0 (256x512), b0, W1, b1, W2, b2, W3, b3], W_l stored [in][out]
    float* w = nullptr;       // FP32 master
    float* g = nullptr;       // gradients
    float* m1 = nullptr;      // Adam first moment
    float* m2 = nullptr;      // Adam second moment
    uint16_t* wf = nullptr;   // BF16 weights, forward layout (NPACK)
    uint16_t* wbk = nullptr;  // BF16 weights, backward layout (NPACK)
    // per batch row (cap_batch rows; the transposed operands padded to whole DW_BK rows)
    uint16_t* ht[NL] = {};    // layer inputs H_0..H_3, transposed [WIDTH[l]][rows]
    uint16_t* gt[NL] = {};    // gradients of the layer outputs G_0..G_3, transposed [NPAD[l]][rows]
    uint16_t* x0 = nullptr;   // features of a predicted batch [256]
    float* out = nullptr;     // network outputs [18]
    float* loss = nullptr;    // [1]
    float* gpart = nullptr;   // [DW_SLICES][NPARAM] partial weight gradients
    float* trace = nullptr;   // [B][MAX_T_GEN] generated traces
    uint64_t* counter = nullptr;  // device step counter for data generation (graph-replay safe)
    // training data ring: GEN_BATCHES consecutive batches generated in one launch
    uint16_t* ring_feat = nullptr;  // [GEN_BATCHES][ring_cap][256]
    float* ring_tgt = nullptr;      // [GEN_BATCHES][ring_cap][18]
    float* ring_trace = nullptr;    // [GEN_BATCHES][ring_cap][MAX_T_GEN]
    int ring_cap = 0;
    opmm_rt::StreamOrder order;  // orders calls on different streams (activations, gradients, Adam state)
};

namespace {

constexpr int MAX_T_GEN = 160;
constexpr int GEN_BATCHES = 16;  // training batches generated per launch (one lane per saccade each)

__global__ void fill_f32_kernel(float* p, int64_t n, float v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// FP32 master weights -> both BF16 layouts (zero padding included), one packed element per thread.
__global__ void pack_weights_kernel(const float* __restrict__ w, uint16_t* __restrict__ wf, uint16_t* __restrict__ wbk)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPACK) return;
    int l = 0;
    while (l < NL - 1 && i >= wpack_off(l + 1)) ++l;
    const int64_t off = i - wpack_off(l);
    const int K = WIDTH[l], N = WIDTH[l + 1];
    const int n = (int)(off / K), k = (int)(off % K);
    const uint16_t h = n < N ? f2bf(w[w_off_c(l) + (int64_t)k * N + n]) : (uint16_t)0;
    wf[wf_index(l, k, n)] = h;
    wbk[wb_index(l, k, n)] = h;
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

// Adam step over every parameter on the stored gradients (the same update the fused weight-gradient
// kernel applies); b1, b2 and their complements om1 = 1 - b1, om2 = 1 - b2 are each the FP32 value
// nearest the exact constant, and c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t) are formed on the host in
// FP64: 1 - b2^t taken in FP32 loses about five digits to cancellation in the first steps.
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                            float* __restrict__ m2, uint16_t* __restrict__ wf, uint16_t* __restrict__ wbk,
                            AdamArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    int l = 0;
    while (l < NL - 1 && i >= w_off_c(l + 1)) ++l;
    const int64_t off = i - w_off_c(l);
    const int N = WIDTH[l + 1];
    const bool is_w = i < b_off_c(l);
    adam_update(i, g[i], w, m1, m2, a, wf, wbk, is_w ? l : -1, is_w ? (int)(off / N) : 0, is_w ? (int)(off % N) : 0);
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
        if (sg->ht[l]) (void)hipFree(sg->ht[l]);
        if (sg->gt[l]) (void)hipFree(sg->gt[l]);
        sg->ht[l] = sg->gt[l] = nullptr;
    }
    for (void* p : {(void*)sg->x0, (void*)sg->out, (void*)sg->trace})
        if (p) (void)hipFree(p);
    sg->x0 = nullptr;
    sg->out = sg->trace = nullptr;
    const size_t rows = (size_t)(batch + DW_BK - 1) / DW_BK * DW_BK;
    for (int l = 0; l < NL; ++l) {
        SG_HIP(hipMalloc(&sg->ht[l], sizeof(uint16_t) * rows * WIDTH[l]));
        SG_HIP(hipMalloc(&sg->gt[l], sizeof(uint16_t) * rows * NPAD[l]));
    }
    SG_HIP(hipMalloc(&sg->x0, sizeof(uint16_t) * (size_t)batch * WIDTH[0]));
    SG_HIP(hipMalloc(&sg->out, sizeof(float) * (size_t)batch * WIDTH[NL]));
    SG_HIP(hipMalloc(&sg->trace, sizeof(float) * (size_t)batch * MAX_T_GEN));
    sg->cap_batch = batch;
    return OPMM_OK;
}

}  // namespace

namespace opmm_rt {
int surrogate_reserve(opmm_surrogate* sg, int batch) { return sg_alloc(sg, batch); }
}  // namespace opmm_rt

namespace {

MlpArgs mlp_args(opmm_surrogate* sg, int B, const uint16_t* x0)
{
    MlpArgs A;
    std::memset(&A, 0, sizeof A);
    A.B = B;
    A.x0 = x0;
    A.wf = sg->wf;
    A.wbk = sg->wbk;
    A.w = sg->w;
    A.Bp = (B + DW_BK - 1) / DW_BK * DW_BK;
    for (int l = 0; l < NL; ++l) {
        A.ht[l] = sg->ht[l];
        A.gt[l] = sg->gt[l];
    }
    return A;
}

// network outputs of the B rows of x0 into out [B][18]: one launch
int sg_forward(opmm_surrogate* sg, int B, const uint16_t* x0, float* out, hipStream_t st)
{
    MlpArgs A = mlp_args(sg, B, x0);
    A.out = out;
    hipLaunchKernelGGL(mlp_pass_kernel<false>, dim3((B + FR - 1) / FR), dim3(FTHREADS), 0, st, A);
    SG_HIP(hipGetLastError());
    return OPMM_OK;
}

AdamArgs adam_args(opmm_surrogate* sg, float lr)
{
    const double b1 = 0.9, b2 = 0.999;
    sg->step += 1;
    AdamArgs a;
    a.lr = lr;
    a.b1 = (float)b1;
    a.om1 = (float)(1.0 - b1);
    a.b2 = (float)b2;
    a.om2 = (float)(1.0 - b2);
    a.eps = 1e-8f;
    a.c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)sg->step)));
    a.c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)sg->step)));
    return a;
}

// Forward, MSE against tgt [B][18] (added to *loss, zeroed by the caller) and backward over the B
// rows of x0: gradients into sg->g.  ADAM: also the Adam step with learning rate lr, and one bump of
// the data-generation counter.  Three launches.
template <bool ADAM>
int sg_step(opmm_surrogate* sg, int B, const uint16_t* x0, const float* tgt, float* loss, float lr, hipStream_t st)
{
    MlpArgs A = mlp_args(sg, B, x0);
    A.target = tgt;
    A.loss = loss;
    // blocks up to Bp: those past the batch write the zero rows of the transposed operands
    hipLaunchKernelGGL(mlp_pass_kernel<true>, dim3(A.Bp / FR), dim3(FTHREADS), 0, st, A);
    SG_HIP(hipGetLastError());
    DwOperands ops;
    for (int l = 0; l < NL; ++l) {
        ops.ht[l] = sg->ht[l];
        ops.gt[l] = sg->gt[l];
    }
    hipLaunchKernelGGL(mlp_dw_kernel, dim3(DW_SLICES * DW_BLOCKS), dim3(256), 0, st, A.Bp, ops, sg->gpart);
    SG_HIP(hipGetLastError());
    AdamArgs a;
    std::memset(&a, 0, sizeof a);
    if (ADAM) a = adam_args(sg, lr);
    hipLaunchKernelGGL(grad_reduce_kernel<ADAM>, dim3(blocks(NPARAM, 256)), dim3(256), 0, st, sg->gpart, sg->g, sg->w,
                       sg->m1, sg->m2, sg->wf, sg->wbk, a, ADAM ? sg->counter : nullptr);
    SG_HIP(hipGetLastError());
    return OPMM_OK;
}

int sg_adam(opmm_surrogate* sg, float lr, hipStream_t st)
{
    const AdamArgs a = adam_args(sg, lr);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, st, sg->w, sg->g, sg->m1, sg->m2, sg->wf,
                       sg->wbk, a);
    return hipGetLastError() == hipSuccess ? OPMM_OK : OPMM_EDEVICE;
}

int sg_pack(opmm_surrogate* sg, hipStream_t st)
{
    hipLaunchKernelGGL(pack_weights_kernel, dim3(blocks(NPACK, 256)), dim3(256), 0, st, sg->w, sg->wf, sg->wbk);
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
        hipMalloc(&sg->wf, sizeof(uint16_t) * NPACK) != hipSuccess ||
        hipMalloc(&sg->wbk, sizeof(uint16_t) * NPACK) != hipSuccess || hipMalloc(&sg->loss, sizeof(float)) != hipSuccess ||
        hipMalloc(&sg->gpart, sizeof(float) * DW_SLICES * NPARAM) != hipSuccess ||
        hipMalloc(&sg->counter, sizeof(uint64_t)) != hipSuccess || opmm_rt::order_init(sg->order) != hipSuccess)
        rc = OPMM_ENOMEM;
    if (rc == OPMM_OK) {
        hipLaunchKernelGGL(init_params_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, 0, sg->w, init_seed);
        hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, 0, sg->m1, NPARAM, 0.0f);
        hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, 0, sg->m2, NPARAM, 0.0f);
        hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks(NPARAM, 256)), dim3(256), 0, 0, sg->g, NPARAM, 0.0f);
        if (sg_pack(sg, 0) != OPMM_OK || hipMemset(sg->counter, 0, sizeof(uint64_t)) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess)
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
        if (sg->ht[l]) (void)hipFree(sg->ht[l]);
        if (sg->gt[l]) (void)hipFree(sg->gt[l]);
    }
    for (void* p : {(void*)sg->w, (void*)sg->g, (void*)sg->m1, (void*)sg->m2, (void*)sg->wf, (void*)sg->wbk,
                    (void*)sg->x0, (void*)sg->out, (void*)sg->loss, (void*)sg->gpart, (void*)sg->trace,
                    (void*)sg->counter,
                    (void*)sg->ring_feat, (void*)sg->ring_tgt, (void*)sg->ring_trace})
        if (p) (void)hipFree(p);
    opmm_rt::order_release(sg->order);
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
    if (sg_pack(sg, 0) != OPMM_OK) return opmm_rt::fail(sg->ctx, OPMM_EDEVICE, "weight packing failed");
    SG_HIP(hipDeviceSynchronize());
    return OPMM_OK;
}

int opmm_surrogate_forward(opmm_surrogate* sg, const uint16_t* feat, int32_t B, float* out, void* stream)
{
    if (!sg || B < 0 || (B > 0 && (!feat || !out))) return OPMM_EINVAL;
    if (B == 0) return OPMM_OK;
    SG_HIP(hipSetDevice(sg->device));
    opmm_rt::Ordered ord(sg->order, (hipStream_t)stream);
    SG_HIP(ord.error());
    return sg_forward(sg, B, feat, out, (hipStream_t)stream);
}

int opmm_surrogate_backward(opmm_surrogate* sg, const uint16_t* feat, const float* target, int32_t B, float* loss_out,
                            void* stream)
{
    if (!sg || B <= 0 || !feat || !target) return OPMM_EINVAL;
    SG_HIP(hipSetDevice(sg->device));
    hipStream_t st = (hipStream_t)stream;
    opmm_rt::Ordered ord(sg->order, st);
    SG_HIP(ord.error());
    int rc;
    if ((rc = sg_alloc(sg, B)) != OPMM_OK) return rc;
    // the pass adds the batch's loss into sg->loss, which only a call that returns it reads: reset it then
    if (loss_out) hipLaunchKernelGGL(fill_f32_kernel, dim3(1), dim3(64), 0, st, sg->loss, 1, 0.0f);
    if ((rc = sg_step<false>(sg, B, feat, target, sg->loss, 0.0f, st)) != OPMM_OK) return rc;
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
    opmm_rt::Ordered ord(sg->order, st);
    SG_HIP(ord.error());
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
    opmm_rt::Ordered ord(sg->order, st);
    SG_HIP(ord.error());
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
        // cosine decay from lr0 to lr_min over this call's steps
        const double ph = n_steps > 1 ? (double)t / (double)(n_steps - 1) : 1.0;
        const float lr = (float)(lr_min + 0.5 * (lr0 - lr_min) * (1.0 + std::cos(M_PI * ph)));
        // forward + loss + backward + Adam (and the counter bump): three launches
        rc = sg_step<true>(sg, B, x0, tgt, hist + t, lr, st);
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
    opmm_rt::Ordered ord(sg->order, (hipStream_t)stream);
    SG_HIP(ord.error());
    return sg_adam(sg, lr, (hipStream_t)stream);
}

// Learned OPC of S uploaded and projected saccades: features, network, de-normalisation into the
// search box.
static int sg_predict(opmm_surrogate* sg, int32_t S, const opmm_rt::SacDev* sd, const float* proj, float dt_ms,
                      float box_frac, float* opc_out, hipStream_t st)
{
    int rc;
    if ((rc = sg_alloc(sg, S)) != OPMM_OK) return rc;
    hipLaunchKernelGGL(features_kernel, dim3(S), dim3(64), 0, st, S, sd, proj, dt_ms, sg->x0);
    if ((rc = sg_forward(sg, S, sg->x0, sg->out, st)) != OPMM_OK) return rc;
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
    opmm_rt::Ordered ord(sg->order, st);
    SG_HIP(ord.error());
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
    opmm_rt::Ordered ord_ctx(opmm_rt::ctx_order(ctx), st);
    SG_HIP(ord_ctx.error());
    opmm_rt::Ordered ord(sg->order, st);
    SG_HIP(ord.error());
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
    opmm_rt::Ordered ord_ctx(opmm_rt::ctx_order(ctx), st);
    SG_HIP(ord_ctx.error());
    opmm_rt::Ordered ord(sg->order, st);
    SG_HIP(ord.error());
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
    opmm_rt::Ordered ord_ctx(opmm_rt::ctx_order(ctx), st);
    SG_HIP(ord_ctx.error());
    opmm_rt::Ordered ord(sg->order, st);
    SG_HIP(ord.error());
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
    if (sg_pack(sg, 0) != OPMM_OK) return opmm_rt::fail(sg->ctx, OPMM_EDEVICE, "weight packing failed");
    SG_HIP(hipDeviceSynchronize());
    sg->step = hdr[1];
    return OPMM_OK;
}

}  // extern "C"
