// policy_tile.h -- one 16-agent tile of the shared policy network on the
// gfx950 matrix cores, used by the policy kernels (policy_mfma.hip) and by the
// view sweep when the policy runs inside the step (flock_kernels.hip).
//
// Sec. 4.3 of arXiv:2207.03945: one policy shared by every agent, so the batch
// axis is the agent axis; Sec. 5: two hidden layers of 64 units.  Network:
// in -> 64 -> 64 -> 2, tanh after every layer.
//
// Precision: inputs, weights and both hidden layers' activations rounded once
// to BF16 (round to nearest even), products accumulated in FP32 by
// v_mfma_f32_16x16x32_bf16 starting from the FP32 biases; tanh evaluated in
// FP32 as 1 - 2 / (exp(2x) + 1) (absolute error about 1e-7).
//
// Layout.  A wave computes the transposed products H1^T = W1^T X^T,
// H2^T = W2^T H1^T and Z^T = W3^T H2^T (units as MFMA rows, agents as
// columns).  Lane l = 16 g + col holds agent col; in register r of output
// tile t (units 16 t .. 16 t + 15) it holds unit 16 t + 4 g + r, and as a B
// operand it supplies the eight K values 32 c + 8 g .. + 7 of chunk c.  Each
// layer's activations reach the next layer's B operand through a per-wave
// LDS tile of BF16 rows; the weights are packed into A-operand lane order
// once on the host (the output layer's two rows padded to 16 with zeros).
//
// Every caller evaluates a tile through mlp_tile and pol_output, so the same
// inputs give bitwise the same actions wherever the network runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

namespace flock {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kHidden = 64;
constexpr int kHidLd = 72;  // BF16 per agent row of the hidden tile (64 + 8 pad)

// Device workspace of one network.
struct PolLayout {
    // A operands, lane (g = l / 16, col = l % 16), element j of chunk c, tile t:
    bf16x8 *w1;  // [kc][4 tiles][64 lanes]  W1[32 c + 8 g + j][16 t + col] (0 beyond in_dim)
    bf16x8 *w2;  // [2][4 tiles][64 lanes]   W2[32 c + 8 g + j][16 t + col]
    bf16x8 *w3;  // [2][64 lanes]            W3[32 c + 8 g + j][col] (0 for col >= outputs)
    float *b1;   // [64] by hidden unit
    float *b2;   // [64]
    float *b3;   // [4]: the outputs' biases, zero-padded
    size_t bytes;
};

// Network biases a block keeps in LDS.
struct alignas(16) PolConsts {
    float b1[64], b2[64], b3[4];
};

__device__ __forceinline__ void load_pol_consts(const PolLayout &P, PolConsts *c, int tid,
                                                int nthreads) {
    for (int i = tid; i < 64; i += nthreads) {
        c->b1[i] = P.b1[i];
        c->b2[i] = P.b2[i];
    }
    if (tid < 4) c->b3[tid] = P.b3[tid];
}

// tanh(x) = 1 - 2 / (exp(2x) + 1): exact limits +-1 when exp overflows or
// underflows, absolute error about 1e-7 (the subtraction from 1).
__device__ __forceinline__ float tanh_fast(float x) {
    const float e = __expf(2.0f * x);
    return __builtin_fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

// Bias of accumulator register r of output tile t (units 16 t + 4 g + r).
__device__ __forceinline__ f32x4 bias4(const float *b, int t, int g) {
    return *reinterpret_cast<const f32x4 *>(b + 16 * t + 4 * g);
}

// Orders a wave's own LDS accesses (lanes of one wave write, then read, a
// tile only that wave uses): a wave's LDS operations complete in issue order,
// so this only keeps the compiler from moving accesses across it (a
// workgroup-scope fence would also wait for the wave's outstanding global
// stores).
__device__ __forceinline__ void wave_lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// tanh of a tile's accumulators, rounded to BF16 into the wave's hidden tile
// as B operand rows of the next layer.
template <class HR>
__device__ __forceinline__ void store_hidden(const f32x4 (&acc)[4], HR hrow, int g, int col) {
    wave_lds_fence();  // earlier reads of the hidden tile come first
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        __bf16 hv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) hv[r] = (__bf16)tanh_fast(acc[t][r]);
        uint2 packed;
        memcpy(&packed, hv, sizeof(packed));
        *reinterpret_cast<uint2 *>(hrow(col) + 16 * t + 4 * g) = packed;
    }
    wave_lds_fence();  // the wave's hidden tile before its reads
}

// One tile of 16 agents through the network.  xb(c): this lane's B operand of
// input chunk c (eight BF16 inputs 32 c + 8 g .. + 7 of agent col, zero beyond
// the input length); w1(c, t), w2(c, t), w3(c): the layers' A operands;
// hrow(col): row col of the wave's hidden tile in LDS, 64 BF16 starting
// 16-byte aligned.  Returns the output pre-activations (z0, z1), biases
// included, in the lanes with g == 0.
template <class XB, class W1, class W2, class W3, class HR>
__device__ __forceinline__ float2 mlp_tile(int kc, XB xb, W1 w1, W2 w2, W3 w3, const PolConsts &pc,
                                          HR hrow, int lane) {
    const int g = lane >> 4, col = lane & 15;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = bias4(pc.b1, t, g);
    for (int c = 0; c < kc; ++c) {
        const bf16x8 x = xb(c);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1(c, t), x, acc[t], 0, 0, 0);
    }
    store_hidden(acc, hrow, g, col);
    bf16x8 hb[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
        hb[c] = *reinterpret_cast<const bf16x8 *>(hrow(col) + 32 * c + 8 * g);
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = bias4(pc.b2, t, g);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2(c, t), hb[c], acc[t], 0, 0, 0);
    store_hidden(acc, hrow, g, col);
#pragma unroll
    for (int c = 0; c < 2; ++c)
        hb[c] = *reinterpret_cast<const bf16x8 *>(hrow(col) + 32 * c + 8 * g);
    f32x4 z = g == 0 ? *reinterpret_cast<const f32x4 *>(pc.b3) : f32x4{};
#pragma unroll
    for (int c = 0; c < 2; ++c) z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3(c), hb[c], z, 0, 0, 0);
    return make_float2(z[0], z[1]);
}

// The actor's action from the output pre-activations: the mean, tanh-squashed
// and scaled to (max_turn, max_dspeed); with kSample, plus sigma * eps, and
// the log density of the sample into *logp (when logp is not null).
template <bool kSample>
__device__ __forceinline__ float2 pol_output(float2 z, float max_turn, float max_dspeed, float2 eps,
                                             float sig0, float sig1, float logp_c, float *logp) {
    float2 a = make_float2(max_turn * tanh_fast(z.x), max_dspeed * tanh_fast(z.y));
    if constexpr (kSample) {
        a.x = a.x + sig0 * eps.x;
        a.y = a.y + sig1 * eps.y;
        if (logp) *logp = -0.5f * (eps.x * eps.x + eps.y * eps.y) + logp_c;
    }
    return a;
}

}  // namespace flock
