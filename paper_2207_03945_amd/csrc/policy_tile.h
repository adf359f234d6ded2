// policy_tile.h -- one 16-agent tile of the shared policy network on the
// gfx950 matrix cores, used by the policy kernels (policy_mfma.hip) and by the
// view sweep when the policy runs inside the step (flock_kernels.hip).
//
// Sec. 4.3 of arXiv:2207.03945: one policy shared by every agent, so the batch
// axis is the agent axis; Sec. 5: two hidden layers of 64 units.  Network:
// in -> 64 -> 64 -> 2, tanh after every layer.
//
// Precision: inputs and weights rounded once to BF16 (round to nearest even),
// products accumulated in FP32 by v_mfma_f32_16x16x32_bf16, biases and the
// 64 -> 2 output layer in FP32 on the vector ALUs (with BF16-rounded weights).
//
// Layout.  A wave computes the transposed products H1^T = W1^T X^T and
// H2^T = W2^T H1^T (hidden units as MFMA rows, agents as columns).  Lane
// l = 16 g + col holds agent col; in register r of output tile t (hidden units
// 16 t .. 16 t + 15) it holds unit 16 t + 4 g + r, and as a B operand it
// supplies the eight K values 32 c + 8 g .. + 7 of chunk c.  Layer 1's
// results reach layer 2 through a per-wave LDS tile of BF16 hidden rows; the
// weights are packed into A-operand lane order once on the host.
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
    float *b1;   // [64] by hidden unit
    float *b2;   // [64]
    float *w3;   // [2 outputs][64] (BF16-rounded)
    float *b3;   // [2]
    size_t bytes;
};

// Network constants a block keeps in LDS.
struct PolConsts {
    float b1[64], b2[64], w3[128], b3[2];
};

__device__ __forceinline__ void load_pol_consts(const PolLayout &P, PolConsts *c, int tid,
                                                int nthreads) {
    for (int i = tid; i < 64; i += nthreads) {
        c->b1[i] = P.b1[i];
        c->b2[i] = P.b2[i];
    }
    for (int i = tid; i < 128; i += nthreads) c->w3[i] = P.w3[i];
    if (tid < 2) c->b3[tid] = P.b3[tid];
}

__device__ __forceinline__ float tanh_fast(float x) {
    x = fminf(fmaxf(x, -15.0f), 15.0f);
    const float e = __expf(2.0f * x);
    return __fdividef(e - 1.0f, e + 1.0f);
}

// One tile of 16 agents through the two hidden layers and the output layer's
// products.  xb(c): this lane's B operand of input chunk c (eight BF16 inputs
// 32 c + 8 g .. + 7 of agent col, zero beyond the input length); w1(c, t) and
// w2(c, t): the layer-1 and layer-2 A operands of chunk c, tile t; s_hid: the
// wave's [16][kHidLd] BF16 hidden tile.  Returns the two output
// pre-activations without bias (z0, z1), summed over the lane groups, in
// every lane.
template <class XB, class W1, class W2>
__device__ __forceinline__ float2 mlp_tile(int kc, XB xb, W1 w1, W2 w2, const PolConsts &pc,
                                          __bf16 *s_hid, int lane) {
    const int g = lane >> 4, col = lane & 15;
    f32x4 acc1[4] = {f32x4{}, f32x4{}, f32x4{}, f32x4{}};
    for (int c = 0; c < kc; ++c) {
        const bf16x8 x = xb(c);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc1[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1(c, t), x, acc1[t], 0, 0, 0);
    }
    // bias + tanh, into the hidden tile as B operand rows of layer 2
    __threadfence_block();  // the previous tile's reads of the hidden tile come first
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        __bf16 hv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) hv[r] = (__bf16)tanh_fast(acc1[t][r] + pc.b1[16 * t + 4 * g + r]);
        uint2 packed;
        memcpy(&packed, hv, sizeof(packed));
        *reinterpret_cast<uint2 *>(s_hid + col * kHidLd + 16 * t + 4 * g) = packed;
    }
    __threadfence_block();  // the wave's hidden tile before its reads
    f32x4 acc2[4] = {f32x4{}, f32x4{}, f32x4{}, f32x4{}};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const bf16x8 hb = *reinterpret_cast<const bf16x8 *>(s_hid + col * kHidLd + 32 * c + 8 * g);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc2[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2(c, t), hb, acc2[t], 0, 0, 0);
    }
    float z0 = 0.0f, z1 = 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int h = 16 * t + 4 * g + r;
            const float hv = tanh_fast(acc2[t][r] + pc.b2[h]);
            z0 = z0 + hv * pc.w3[h];
            z1 = z1 + hv * pc.w3[64 + h];
        }
    z0 = z0 + __shfl_xor(z0, 16, 64);
    z1 = z1 + __shfl_xor(z1, 16, 64);
    z0 = z0 + __shfl_xor(z0, 32, 64);
    z1 = z1 + __shfl_xor(z1, 32, 64);
    return make_float2(z0, z1);
}

// The actor's action from the output pre-activations: the mean, tanh-squashed
// and scaled to (max_turn, max_dspeed); with kSample, plus sigma * eps, and
// the log density of the sample into *logp (when logp is not null).
template <bool kSample>
__device__ __forceinline__ float2 pol_output(float2 z, const PolConsts &pc, float max_turn,
                                             float max_dspeed, float2 eps, float sig0, float sig1,
                                             float logp_c, float *logp) {
    float2 a = make_float2(max_turn * tanhf(z.x + pc.b3[0]), max_dspeed * tanhf(z.y + pc.b3[1]));
    if constexpr (kSample) {
        a.x = a.x + sig0 * eps.x;
        a.y = a.y + sig1 * eps.y;
        if (logp) *logp = -0.5f * (eps.x * eps.x + eps.y * eps.y) + logp_c;
    }
    return a;
}

}  // namespace flock
