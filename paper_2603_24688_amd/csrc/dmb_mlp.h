// dmb_mlp.h -- learned closure for the rate integrals of eq. scrA / scrB.
//
// For sigma-bar = sigma0 (v/c)^n the gas pass needs, per pair,
//   Ahat / vs^{n+1} = (alpha_n/3) 1F1(-(n+1)/2, 5/2, -u^2/2),
//   Bhat / vs^{n+3} =  alpha_n    1F1(-(n+3)/2, 3/2, -u^2/2),   u = w / vs
// (Appendix B).  A 3 x 64 ReLU network predicts the logarithm of both terms
// relative to base functions a(u) = (c0 + c1 u^2 + u^4)^{p/4} (p = n+1 for A,
// n+3 for B; c0 makes a(0) the u = 0 value, the u^p tail is the large-w limit
// sigma(w) w, sigma(w) w^3 of the rates; c1 below), from s = 2u/(u+2) - 1 and
// a one-hot code of n.  With a Maxwellian DM population (temperature ratio x2,
// mass ratio 10^{x3}) the same network applies at u = x1 / r,
// r = sqrt(1 + x2 10^{-x3}), with the extra factors r^{n+1}, r^{n+3}.
//
// Arithmetic: bfloat16 MFMA with binary32 accumulation.  All four layers run
// on v_mfma_f32_16x16x{16,32}_bf16; the output of one layer is the B operand
// of the next without leaving registers: in the 16x16 D layout lane l holds
// rows 4(l/16)+i (i = 0..3) of column l%16, and the B operand of the next
// 16x16x32 product wants contraction indices 8(l/16)+j (j = 0..7) of the same
// column.  Reading the packed D registers of two neighbouring 16-row blocks as
// one B fragment therefore contracts over a fixed permutation of the hidden
// units, nu(kappa) below, which the packed weights absorb.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dmb_device.h"

namespace dmb {

constexpr int kMlpH = 64;              // hidden units per layer
constexpr int kMlpIn = 5;              // s and one-hot(n)
constexpr int kMlpOut = 2;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpH * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpH * kMlpH;
constexpr int kOffW4 = kOffB3 + kMlpH;
constexpr int kOffB4 = kOffW4 + kMlpOut * kMlpH;
constexpr int kMlpParams = kOffB4 + kMlpOut;   // 8834
constexpr float kMlpTScale = 2.f;              // s = 2u/(u + kMlpTScale) - 1
constexpr float kMlpUMax = 1000.f;             // trained range of u
constexpr float kMlpLossScale = 10.f;          // L = scale^2 sum (o - y)^2 / (2B)
constexpr int kMlpWave = 64;                   // samples per wave (4 column blocks of 16)
// Shape constants c1 of the base functions, [n index][A, B]: the values (3
// decimals) minimising the largest |residual| over 0 <= u <= 1000.
constexpr double kMlpC1[4][2] = {{0.833, 0.694}, {4.327, 4.114}, {8.061, 7.967}, {11.981, 12.089}};

__host__ __device__ constexpr int mlp_n_index(int n)
{
    return n == -4 ? 0 : n == -2 ? 1 : n == 0 ? 2 : n == 2 ? 3 : -1;
}

// Contraction index kappa (0..63) of a chained 16x16x32 product -> hidden unit.
__host__ __device__ constexpr int mlp_nu(int kappa)
{
    const int s = kappa >> 5, h = (kappa >> 3) & 3, j = kappa & 7;
    return 16 * (2 * s + (j >> 2)) + 4 * h + (j & 3);
}
// Inverse of mlp_nu.
__host__ __device__ constexpr int mlp_kappa(int nu)
{
    const int blk = nu >> 4, s = blk >> 1, jh = blk & 1, h = (nu >> 2) & 3, jl = nu & 3;
    return 32 * s + 8 * h + 4 * jh + jl;
}

// Packed weights.  The first part (through b4) is what inference reads; the
// transposed copies serve the backward pass.  bfloat16 values are stored as
// raw 16-bit patterns.
struct MlpBlob {
    uint16_t w1[kMlpH][16];       // [unit][slot]: slots (w_s, w_s, w_n0..w_n3, 0 ...)
    float b1[kMlpH];
    uint16_t w2[kMlpH][kMlpH];    // [out unit][kappa] = W2[out][nu(kappa)]
    float b2[kMlpH];
    uint16_t w3[kMlpH][kMlpH];
    float b3[kMlpH];
    uint16_t w4[16][kMlpH];       // rows 0, 1 = outputs; rows 2..15 zero
    float b4[16];
    uint16_t w2t[kMlpH][kMlpH];   // [in unit][kappa] = W2[nu(kappa)][in]
    uint16_t w3t[kMlpH][kMlpH];
    float w4f[kMlpOut][kMlpH];    // bfloat16-rounded W4 as binary32
};
constexpr size_t kMlpInferBytes = offsetof(MlpBlob, w2t);

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// binary32 -> bfloat16 bits, round to nearest even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t bf16_pack2(float a, float b)
{
    f32x2 f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
}
__device__ __forceinline__ uint16_t bf16_bits(float a) { return uint16_t(bf16_pack2(a, 0.f) & 0xFFFFu); }
__device__ __forceinline__ float bf16_float(uint32_t bits16) { return __uint_as_float(bits16 << 16); }
__device__ __forceinline__ float bf16_round(float a) { return bf16_float(bf16_bits(a)); }

// ReLU then bfloat16 for two values: the sign bit of a bfloat16 is the sign
// of its 16-bit integer pattern, so a packed signed max with 0 is the ReLU.
__device__ __forceinline__ uint32_t relu_pack2(float a, float b)
{
    s16x2 s = __builtin_bit_cast(s16x2, bf16_pack2(a, b));
    s16x2 z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(s, z));
}

__device__ __forceinline__ f32x4 mfma32(uint4 a, uint4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(uint2 a, uint2 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a), __builtin_bit_cast(s16x4, b), c,
                                                     0, 0, 0);
}

// Pack the D fragments of blocks 2s and 2s+1 (ReLU, bfloat16) into the B
// operand of contraction step s.
__device__ __forceinline__ uint4 act_frag(f32x4 lo, f32x4 hi)
{
    return make_uint4(relu_pack2(lo[0], lo[1]), relu_pack2(lo[2], lo[3]), relu_pack2(hi[0], hi[1]),
                      relu_pack2(hi[2], hi[3]));
}

// Layer-1 B operand of one column: slots (s_hi, s_lo, onehot(n)) split over
// lane groups h = 0 (slots 0..3) and h = 1 (slots 4..7).
__device__ __forceinline__ uint2 input_frag(float s, int nidx, int h)
{
    const uint32_t hi16 = bf16_bits(s);
    const float lo = s - bf16_float(hi16);
    const uint32_t lo16 = bf16_bits(lo);
    const uint32_t one = 0x3F80u;
    if (h == 0)
        return make_uint2(hi16 | (lo16 << 16), (nidx == 0 ? one : 0u) | ((nidx == 1 ? one : 0u) << 16));
    if (h == 1) return make_uint2((nidx == 2 ? one : 0u) | ((nidx == 3 ? one : 0u) << 16), 0u);
    return make_uint2(0u, 0u);
}

// Network input s = 2u/(u+2) - 1.
__device__ __forceinline__ float mlp_input(float u) { return 2.f * u / (u + kMlpTScale) - 1.f; }

// Forward pass of one wave over 64 columns (column = lane), weights read from
// `W` (LDS or global).  Column c of block b is lane 16b + c.  Returns the two
// network outputs of the lane's own column.  All 64 lanes must be active.
// The four column blocks go through the layers NB at a time (NB = 4 loads
// each weight fragment once; NB = 2 halves the live accumulators).
// If `act` is non-null the bfloat16 activations of layers 1..3 are kept
// there: act[layer][block][step] (B-operand layout of the lane).
// NBLK < 4 evaluates only the first NBLK column blocks (lanes 0 .. 16 NBLK - 1);
// the other lanes return 0.
template <int NB = 4, int NBLK = 4>
__device__ __forceinline__ void mlp_forward64(const MlpBlob* __restrict__ W, float s_in, int nidx, float* yA,
                                              float* yB, uint4 (*act)[4][2] = nullptr)
{
    static_assert(NB == 1 || NB == 2 || NB == 4, "column blocks per round");
    const int l = threadIdx.x & 63, h = l >> 4, c = l & 15;
    float oA = 0.f, oB = 0.f;
#pragma unroll 1
    for (int r = 0; r < (NBLK + NB - 1) / NB; ++r) {
        f32x4 D[NB][4];
        uint4 Bx[NB][2];
        // layer 1 (16x16x16): four 16-unit blocks
        uint2 B1[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b)
            B1[b] = input_frag(__shfl(s_in, 16 * (NB * r + b) + c), __shfl(nidx, 16 * (NB * r + b) + c), h);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const uint2 A = *reinterpret_cast<const uint2*>(&W->w1[16 * mb + c][4 * h]);
            const f32x4 C = *reinterpret_cast<const f32x4*>(&W->b1[16 * mb + 4 * h]);
#pragma unroll
            for (int b = 0; b < NB; ++b) D[b][mb] = mfma16(A, B1[b], C);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            Bx[b][0] = act_frag(D[b][0], D[b][1]);
            Bx[b][1] = act_frag(D[b][2], D[b][3]);
            if (act) { act[0][NB * r + b][0] = Bx[b][0]; act[0][NB * r + b][1] = Bx[b][1]; }
        }
        // layers 2 and 3 (16x16x32)
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
            const uint16_t(*w)[kMlpH] = layer == 0 ? W->w2 : W->w3;
            const float* bias = layer == 0 ? W->b2 : W->b3;
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const f32x4 C = *reinterpret_cast<const f32x4*>(&bias[16 * mb + 4 * h]);
                const uint4 A0 = *reinterpret_cast<const uint4*>(&w[16 * mb + c][8 * h]);
                const uint4 A1 = *reinterpret_cast<const uint4*>(&w[16 * mb + c][32 + 8 * h]);
#pragma unroll
                for (int b = 0; b < NB; ++b) D[b][mb] = mfma32(A1, Bx[b][1], mfma32(A0, Bx[b][0], C));
                // keep each block's weight reads next to their use (bounds live registers)
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                Bx[b][0] = act_frag(D[b][0], D[b][1]);
                Bx[b][1] = act_frag(D[b][2], D[b][3]);
                if (act) { act[layer + 1][NB * r + b][0] = Bx[b][0]; act[layer + 1][NB * r + b][1] = Bx[b][1]; }
            }
        }
        // output layer: rows 0 and 1 of a 16-row block, read back by the
        // lanes whose own column it is
        const f32x4 C4 = *reinterpret_cast<const f32x4*>(&W->b4[4 * h]);
        const uint4 A0 = *reinterpret_cast<const uint4*>(&W->w4[c][8 * h]);
        const uint4 A1 = *reinterpret_cast<const uint4*>(&W->w4[c][32 + 8 * h]);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const f32x4 O = mfma32(A1, Bx[b][1], mfma32(A0, Bx[b][0], C4));
            const float vA = __shfl(O[0], c), vB = __shfl(O[1], c);
            if (h == NB * r + b) { oA = vA; oB = vB; }
        }
    }
    *yA = oA;
    *yB = oB;
}

// q^{K/4} for the odd K the base functions need.
template <int K>
__device__ __forceinline__ float pow_quarter(float q)
{
    if constexpr (K == 1) return __fsqrt_rn(__fsqrt_rn(q));
    else if constexpr (K == -1) return __frsqrt_rn(__fsqrt_rn(q));
    else if constexpr (K == 3) { const float h = __fsqrt_rn(q); return h * __fsqrt_rn(h); }
    else if constexpr (K == -3) { const float r = __frsqrt_rn(q); return r * __fsqrt_rn(r); }
    else { static_assert(K == 5, "exponent"); return q * __fsqrt_rn(__fsqrt_rn(q)); }
}

// Base functions (n fixed): bA = (c0A + c1A u^2 + u^4)^{(n+1)/4},
// bB = (c0B + c1B u^2 + u^4)^{(n+3)/4}.
template <int N>
__device__ __forceinline__ void mlp_base(float u2, float c0A, float c1A, float c0B, float c1B, float* bA, float* bB)
{
    *bA = pow_quarter<N + 1>(c0A + u2 * (c1A + u2));
    *bB = pow_quarter<N + 3>(c0B + u2 * (c1B + u2));
}


// ---------------------------------------------------------------------------
// Training.  One sample = float4 (s, n index, y_A, y_B) with the residual
// targets y of the two logarithms.

constexpr uint32_t kTagMlpInit = 4u;

// He-uniform initial weights, zero biases, from Philox (counter = (parameter,
// 0, 0, tag 4), key = seed).
__global__ __launch_bounds__(256) void k_mlp_init(float* p, uint32_t k0, uint32_t k1)
{
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i >= kMlpParams) return;
    float fan = 0.f;
    if (i < kOffB1) fan = float(kMlpIn);
    else if ((i >= kOffW2 && i < kOffB2) || (i >= kOffW3 && i < kOffB3) || (i >= kOffW4 && i < kOffB4)) fan = float(kMlpH);
    float v = 0.f;
    if (fan > 0.f) {
        const U4 r = philox_block(uint32_t(i), 0u, 0u, kTagMlpInit, 0u, k0, k1);
        v = (2.f * u24<float>(r.x) - 1.f) * sqrtf(6.f / fan);
    }
    p[i] = v;
}

// Write parameter i of the binary32 vector into every place the packed
// weights hold it.  Entries the packing never writes stay zero.
__device__ __forceinline__ void mlp_pack_one(int i, float v, MlpBlob* B)
{
    const uint16_t q = bf16_bits(v);
    if (i < kOffB1) {
        const int u = i / kMlpIn, k = i % kMlpIn;
        if (k == 0) { B->w1[u][0] = q; B->w1[u][1] = q; }
        else B->w1[u][1 + k] = q;
    } else if (i < kOffW2) {
        B->b1[i - kOffB1] = v;
    } else if (i < kOffB2) {
        const int o = (i - kOffW2) / kMlpH, in = (i - kOffW2) % kMlpH;
        B->w2[o][mlp_kappa(in)] = q;
        B->w2t[in][mlp_kappa(o)] = q;
    } else if (i < kOffW3) {
        B->b2[i - kOffB2] = v;
    } else if (i < kOffB3) {
        const int o = (i - kOffW3) / kMlpH, in = (i - kOffW3) % kMlpH;
        B->w3[o][mlp_kappa(in)] = q;
        B->w3t[in][mlp_kappa(o)] = q;
    } else if (i < kOffW4) {
        B->b3[i - kOffB3] = v;
    } else if (i < kOffB4) {
        const int o = (i - kOffW4) / kMlpH, in = (i - kOffW4) % kMlpH;
        B->w4[o][mlp_kappa(in)] = q;
        B->w4f[o][in] = bf16_float(q);
    } else {
        B->b4[i - kOffB4] = v;
    }
}

__global__ __launch_bounds__(256) void k_mlp_pack(const float* p, MlpBlob* B)
{
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i < kMlpParams) mlp_pack_one(i, p[i], B);
}

// Residual targets by binary64 quadrature of the rate integrals (the
// quadrature of rate_quad, normalised to the 1F1 terms).  x[k] = (x1, x2, x3, n).
struct MlpConst {
    double lnA[4], lnB[4];     // ln(alpha_n/3), ln(alpha_n)
    double c0A[4], c0B[4];     // (alpha_n/3)^{4/(n+1)}, alpha_n^{4/(n+3)}
    double inv_alpha[4];
};

// ln a_A(u), ln a_B(u) in binary64.
__device__ __forceinline__ void mlp_base_logs(double u, int j, int n, const MlpConst& K, double* la, double* lb)
{
    const double u2 = u * u;
    *la = 0.25 * (n + 1) * log(K.c0A[j] + u2 * (kMlpC1[j][0] + u2));
    *lb = 0.25 * (n + 3) * log(K.c0B[j] + u2 * (kMlpC1[j][1] + u2));
}

template <int N>
__device__ __forceinline__ void mlp_label_n(double u, const MlpConst& K, const double* gx, const double* gw, int nq,
                                            double hw, double bmin, double* yA, double* yB)
{
    constexpr int j = mlp_n_index(N);
    double FA, FB, la, lb;
    rate_quad<N, double>(u, gx, gw, nq, K.inv_alpha[j], hw, bmin, &FA, &FB);
    mlp_base_logs(u, j, N, K, &la, &lb);
    *yA = K.lnA[j] + log(FA) - la;
    *yB = K.lnB[j] + log(FB) - lb;
}

__global__ __launch_bounds__(256) void k_mlp_labels(int64_t n, const double* x, MlpConst K, const double* gx,
                                                    const double* gw, int nq, double hw, double bmin, double* y)
{
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k >= n) return;
    const double x1 = x[4 * k], x2 = x[4 * k + 1], x3 = x[4 * k + 2];
    const int nv = int(x[4 * k + 3]);
    const double u = x1 / sqrt(1.0 + x2 * exp10(-x3));
    double a = NAN, b = NAN;
    switch (nv) {
        case -4: mlp_label_n<-4>(u, K, gx, gw, nq, hw, bmin, &a, &b); break;
        case -2: mlp_label_n<-2>(u, K, gx, gw, nq, hw, bmin, &a, &b); break;
        case 0: mlp_label_n<0>(u, K, gx, gw, nq, hw, bmin, &a, &b); break;
        case 2: mlp_label_n<2>(u, K, gx, gw, nq, hw, bmin, &a, &b); break;
    }
    y[2 * k] = a;
    y[2 * k + 1] = b;
}

// Training samples (s, n index, y_A, y_B) from x and binary64 targets.
__global__ __launch_bounds__(256) void k_mlp_prep(int64_t n, const double* x, const double* y, float4* ts)
{
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k >= n) return;
    const double u = x[4 * k] / sqrt(1.0 + x[4 * k + 1] * exp10(-x[4 * k + 2]));
    const float s = float(2.0 * u / (u + double(kMlpTScale)) - 1.0);
    ts[k] = make_float4(s, float(mlp_n_index(int(x[4 * k + 3]))), float(y[2 * k]), float(y[2 * k + 1]));
}

// Network outputs for samples x (binary64 in, log-rates out):
// out = (ln Ahat/vs^{n+1}, ln Bhat/vs^{n+3}).  u > kMlpUMax: quadrature.
__global__ __launch_bounds__(64) void k_mlp_eval(int64_t n, const double* x, const MlpBlob* W, MlpConst K,
                                                 const double* gx, const double* gw, int nq, double hw, double bmin,
                                                 double* out)
{
    const int64_t k = int64_t(blockIdx.x) * 64 + threadIdx.x;
    const bool ok = k < n;
    double u = 0.0, r = 1.0;
    int nv = 0;
    if (ok) {
        r = sqrt(1.0 + x[4 * k + 1] * exp10(-x[4 * k + 2]));
        u = x[4 * k] / r;
        nv = int(x[4 * k + 3]);
    }
    const int j = mlp_n_index(nv);
    const float s = float(2.0 * u / (u + double(kMlpTScale)) - 1.0);
    float oA, oB;
    mlp_forward64(W, s, j < 0 ? 0 : j, &oA, &oB);
    if (!ok) return;
    double yA = oA, yB = oB;
    if (j < 0) {
        yA = yB = NAN;
    } else if (u > double(kMlpUMax)) {
        switch (nv) {
            case -4: mlp_label_n<-4>(u, K, gx, gw, nq, hw, bmin, &yA, &yB); break;
            case -2: mlp_label_n<-2>(u, K, gx, gw, nq, hw, bmin, &yA, &yB); break;
            case 0: mlp_label_n<0>(u, K, gx, gw, nq, hw, bmin, &yA, &yB); break;
            case 2: mlp_label_n<2>(u, K, gx, gw, nq, hw, bmin, &yA, &yB); break;
        }
    }
    const double lr = log(r);
    double la = 0.0, lb = 0.0;
    if (j >= 0) mlp_base_logs(u, j, nv, K, &la, &lb);
    out[2 * k] = (nv + 1) * lr + la + yA;
    out[2 * k + 1] = (nv + 3) * lr + lb + yB;
}

// One minibatch slice of 64 samples per block: forward, loss, backward.
// Writes this block's gradient and loss terms to part[block][0..kMlpParams].
// Sample g of the batch is training sample (mul * (step * batch + g) + add) mod n;
// mul, add come from shuffle[epoch] (identity when shuffle is null).
struct MlpGradArgs {
    const float4* ts; int64_t n_total;
    int64_t batch;              // samples in the minibatch (loss normalisation)
    const uint32_t* epoch;      // device epoch counter (nullable)
    const uint64_t* shuffle;    // [epochs][2] (nullable)
    int64_t step;               // minibatch index within the epoch
    const MlpBlob* W;
    float* part;                // [blocks][kMlpParams + 1]
};

constexpr int kMlpLd = kMlpH + 1;   // padded LDS row

__global__ __launch_bounds__(64) void k_mlp_grad(MlpGradArgs a)
{
    __shared__ float F[3][kMlpWave][kMlpLd];    // activations a1..a3, [sample][unit]
    __shared__ float G[2][kMlpWave][kMlpLd];    // error signals, [sample][unit]
    __shared__ float E[kMlpWave][2], S[kMlpWave];
    __shared__ int NI[kMlpWave];
    const int l = threadIdx.x, h = l >> 4, c = l & 15;
    float* out = a.part + int64_t(blockIdx.x) * (kMlpParams + 1);
    const int64_t g = int64_t(blockIdx.x) * kMlpWave + l;
    const bool ok = g < a.batch;
    float4 smp = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ok) {
        int64_t idx = a.step * a.batch + g;
        if (a.shuffle) {
            const uint64_t* sh = a.shuffle + 2 * (a.epoch ? *a.epoch : 0u);
            idx = int64_t((unsigned __int128)(uint64_t(idx) % uint64_t(a.n_total)) * sh[0] % uint64_t(a.n_total));
            idx = int64_t((uint64_t(idx) + sh[1]) % uint64_t(a.n_total));
        } else {
            idx %= a.n_total;
        }
        smp = a.ts[idx];
    }
    const int nidx = int(smp.y);
    uint4 act[3][4][2];
    float oA, oB;
    mlp_forward64(a.W, smp.x, nidx, &oA, &oB, act);
    // loss terms and output error
    const float ls2 = kMlpLossScale * kMlpLossScale;
    const float rA = ok ? oA - smp.z : 0.f, rB = ok ? oB - smp.w : 0.f;
    float lsum = 0.5f * ls2 * (rA * rA + rB * rB) / float(a.batch);
    for (int d = 32; d >= 1; d >>= 1) lsum += __shfl_xor(lsum, d);
    if (l == 0) out[kMlpParams] = lsum;
    E[l][0] = ls2 * rA / float(a.batch);
    E[l][1] = ls2 * rB / float(a.batch);
    {
        const uint32_t hi16 = bf16_bits(smp.x);
        S[l] = bf16_float(hi16) + bf16_round(smp.x - bf16_float(hi16));
        NI[l] = nidx;
    }
    // activations to [sample][unit]
#pragma unroll
    for (int ly = 0; ly < 3; ++ly)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int st = 0; st < 2; ++st) {
                const uint4 v = act[ly][b][st];
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    F[ly][16 * b + c][mlp_nu(32 * st + 8 * h + j)] = bf16_float((w[j >> 1] >> (16 * (j & 1))) & 0xFFFFu);
            }
    __syncthreads();
    // output layer (lane = unit): dW4, db4, and the layer-3 error
    {
        float g0 = 0.f, g1 = 0.f, db = 0.f;
        const float w0 = a.W->w4f[0][l], w1 = a.W->w4f[1][l];
        for (int b = 0; b < kMlpWave; ++b) {
            const float e0 = E[b][0], e1 = E[b][1], x = F[2][b][l];
            g0 += e0 * x;
            g1 += e1 * x;
            const float d = x > 0.f ? e0 * w0 + e1 * w1 : 0.f;
            G[0][b][l] = d;
            db += d;
        }
        out[kOffW4 + l] = g0;
        out[kOffW4 + kMlpH + l] = g1;
        out[kOffB3 + l] = db;
        if (l < 2) {
            float s = 0.f;
            for (int b = 0; b < kMlpWave; ++b) s += E[b][l];
            out[kOffB4 + l] = s;
        }
    }
    __syncthreads();
    // layers 3 and 2: weight gradient (MFMA over samples), then the error of
    // the layer below (MFMA over units)
#pragma unroll 1
    for (int ly = 1; ly >= 0; --ly) {
        const float(*Gi)[kMlpLd] = G[(1 - ly) & 1];     // error of layer ly+2: ly=1 -> G[0], ly=0 -> G[1]
        float(*Go)[kMlpLd] = G[ly & 1];                 // error of layer ly+1
        const float(*Fin)[kMlpLd] = F[ly];               // input activations of layer ly+2
        const int offW = ly == 1 ? kOffW3 : kOffW2;
        const uint16_t(*wt)[kMlpH] = ly == 1 ? a.W->w3t : a.W->w2t;
        // dW[out][in] = sum_samples q(err[s][out]) act[s][in]
        f32x4 D[4][4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) D[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            uint4 Af[4], Bf[4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                float v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = Gi[32 * st + 8 * h + j][16 * mb + c];
                Af[mb] = make_uint4(bf16_pack2(v[0], v[1]), bf16_pack2(v[2], v[3]), bf16_pack2(v[4], v[5]),
                                    bf16_pack2(v[6], v[7]));
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = Fin[32 * st + 8 * h + j][16 * mb + c];
                Bf[mb] = make_uint4(bf16_pack2(v[0], v[1]), bf16_pack2(v[2], v[3]), bf16_pack2(v[4], v[5]),
                                    bf16_pack2(v[6], v[7]));
            }
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) D[mb][nb] = mfma32(Af[mb], Bf[nb], D[mb][nb]);
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) out[offW + (16 * mb + 4 * h + i) * kMlpH + 16 * nb + c] = D[mb][nb][i];
        // err_below[s][unit] = (sum_k q(W)[k][unit] q(err[s][k])) * [act[s][unit] > 0]
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) D[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            uint4 Bf[4];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                float v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = Gi[16 * nb + c][mlp_nu(32 * st + 8 * h + j)];
                Bf[nb] = make_uint4(bf16_pack2(v[0], v[1]), bf16_pack2(v[2], v[3]), bf16_pack2(v[4], v[5]),
                                    bf16_pack2(v[6], v[7]));
            }
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const uint4 A = *reinterpret_cast<const uint4*>(&wt[16 * mb + c][32 * st + 8 * h]);
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) D[mb][nb] = mfma32(A, Bf[nb], D[mb][nb]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int u = 16 * mb + 4 * h + i, smp_i = 16 * nb + c;
                    Go[smp_i][u] = Fin[smp_i][u] > 0.f ? D[mb][nb][i] : 0.f;
                }
        __syncthreads();
        // bias gradient of layer ly+1 (lane = unit)
        float db = 0.f;
        for (int b = 0; b < kMlpWave; ++b) db += Go[b][l];
        out[(ly == 1 ? kOffB2 : kOffB1) + l] = db;
        __syncthreads();
    }
    // layer 1 weights (lane = unit): inputs (s, one-hot n)
    {
        float gs = 0.f, gn[4] = {0.f, 0.f, 0.f, 0.f};
        for (int b = 0; b < kMlpWave; ++b) {
            const float d = G[0][b][l];
            gs += d * S[b];
            const int k = NI[b];
            gn[0] += k == 0 ? d : 0.f;
            gn[1] += k == 1 ? d : 0.f;
            gn[2] += k == 2 ? d : 0.f;
            gn[3] += k == 3 ? d : 0.f;
        }
        out[kOffW1 + l * kMlpIn] = gs;
        for (int k = 0; k < 4; ++k) out[kOffW1 + l * kMlpIn + 1 + k] = gn[k];
    }
}

// Sum of the block partials (fixed order).
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* part, int nblk, float* out)
{
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (i > kMlpParams) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[int64_t(b) * (kMlpParams + 1) + i];
    out[i] = s;
}

// Adam (Kingma & Ba 2015) on the binary32 master weights with a cosine
// learning rate, then repacking of the bfloat16 weights.  The global step is
// t = epoch * steps_per_epoch + step + 1.
struct MlpAdamArgs {
    float* p; float* m; float* v;
    const float* part; int nblk;
    const uint32_t* epoch; int64_t step, steps_per_epoch, total_steps;
    float lr0, lr_min, beta1, beta2, eps;
    MlpBlob* W;
    float* loss;                // [total_steps]
};

__global__ __launch_bounds__(256) void k_mlp_adam(MlpAdamArgs a)
{
    const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
    const int64_t t = int64_t(a.epoch ? *a.epoch : 0u) * a.steps_per_epoch + a.step + 1;
    if (i == kMlpParams) {
        float s = 0.f;
        for (int b = 0; b < a.nblk; ++b) s += a.part[int64_t(b) * (kMlpParams + 1) + kMlpParams];
        a.loss[t - 1] = s;
        return;
    }
    if (i > kMlpParams) return;
    float g = 0.f;
    for (int b = 0; b < a.nblk; ++b) g += a.part[int64_t(b) * (kMlpParams + 1) + i];
    const float lr = a.lr_min + 0.5f * (a.lr0 - a.lr_min) *
                                    (1.f + cosf(3.14159265358979f * float(t - 1) / float(a.total_steps)));
    const float m = a.beta1 * a.m[i] + (1.f - a.beta1) * g;
    const float v = a.beta2 * a.v[i] + (1.f - a.beta2) * g * g;
    a.m[i] = m;
    a.v[i] = v;
    const float mh = m / (1.f - powf(a.beta1, float(t))), vh = v / (1.f - powf(a.beta2, float(t)));
    const float p = a.p[i] - lr * mh / (sqrtf(vh) + a.eps);
    a.p[i] = p;
    mlp_pack_one(i, p, a.W);
}

__global__ void k_mlp_tick(uint32_t* epoch) { epoch[0] += 1u; }

}  // namespace dmb
