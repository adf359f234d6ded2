// rl_kernels.hip -- trajectory processing over an on-device rollout buffer.
//
// Sec. 4.3 and Fig. 5 of arXiv:2207.03945: every agent is an independent PPO
// learner and the simulation's views and rewards feed the learner's
// experience buffer; Sec. 5: t = 128 simulation updates per training step.
// The advantage of each agent is PPO's truncated estimator over the segment,
// bootstrapped with the value of the state after the last step:
//     delta_t = r_t + gamma V_{t+1} - V_t,   A_t = delta_t + gamma lambda A_{t+1},
//     A_T = 0,   R_t = A_t + V_t.
// One thread per agent walks t backwards; rows t of the [T][n] buffers are
// contiguous over agents, so every load and store is coalesced.  The
// recurrence runs in FP64 and each output is rounded once to FP32.  Loads
// for kChunk steps are issued before the chunk's recurrence, so a wave keeps
// kChunk rows of both inputs in flight (the kernel is HBM-bound: 16 bytes per
// agent-step).
#include <math.h>

#include "flock_internal.h"

namespace flock {

namespace {

constexpr int kGaeBlock = 256;
constexpr int kChunk = 16;

__global__ __launch_bounds__(kGaeBlock) void k_gae(int T, int64_t n, double gamma, double gl,
                                                   const float *__restrict__ rew,
                                                   const float *__restrict__ val,
                                                   float *__restrict__ adv,
                                                   float *__restrict__ ret) {
    const int64_t i = (int64_t)blockIdx.x * kGaeBlock + threadIdx.x;
    if (i >= n) return;
    double a = 0.0;
    double v_next = (double)val[(size_t)T * n + i];
    int t1 = T;  // steps [t1 - kChunk, t1) are next
    for (; t1 >= kChunk; t1 -= kChunk) {
        float r[kChunk], v[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const size_t at = (size_t)(t1 - 1 - u) * n + i;
            r[u] = rew[at];
            v[u] = val[at];
        }
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const size_t at = (size_t)(t1 - 1 - u) * n + i;
            const double vt = (double)v[u];
            a = ((double)r[u] + gamma * v_next - vt) + gl * a;
            adv[at] = (float)a;
            ret[at] = (float)(a + vt);
            v_next = vt;
        }
    }
    for (int t = t1 - 1; t >= 0; --t) {
        const size_t at = (size_t)t * n + i;
        const double vt = (double)val[at];
        a = ((double)rew[at] + gamma * v_next - vt) + gl * a;
        adv[at] = (float)a;
        ret[at] = (float)(a + vt);
        v_next = vt;
    }
}

}  // namespace

}  // namespace flock

using namespace flock;

extern "C" {

int rl_gae(int steps, int64_t n, float gamma, float lambda, const float *reward,
           const float *value, float *adv, float *ret, void *stream) {
    if (steps < 1 || n < 0) return set_error(ENV_EINVAL, "need steps >= 1 and n >= 0");
    if (!(gamma >= 0.0f && gamma <= 1.0f) || !(lambda >= 0.0f && lambda <= 1.0f))
        return set_error(ENV_EINVAL, "gamma and lambda must lie in [0, 1]");
    if (n == 0) return ENV_OK;
    if (!reward || !value || !adv || !ret) return set_error(ENV_EINVAL, "NULL buffer");
    const double g = gamma, gl = (double)gamma * (double)lambda;
    hipLaunchKernelGGL(k_gae, dim3((unsigned)((n + kGaeBlock - 1) / kGaeBlock)), dim3(kGaeBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), steps, n, g, gl, reward, value, adv,
                       ret);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ENV_EHIP, "rl_gae: %s", hipGetErrorString(e));
    return ENV_OK;
}

}  // extern "C"
