// policy_mfma.hip -- the shared policy network on gfx950 matrix cores.
//
// Sec. 4.3 of arXiv:2207.03945: one policy shared by every agent, each agent
// an independent learner, so the batch axis is the agent axis; Sec. 5: two
// hidden layers of 64 units.  Here: in -> 64 -> 64 -> 2, tanh after every
// layer, the two outputs scaled to the turn / speed-change ranges of Sec. 4.1.
//
// Precision: inputs and weights rounded once to BF16 (round to nearest even),
// products accumulated in FP32 by v_mfma_f32_16x16x32_bf16, biases and the
// 64 -> 2 output layer in FP32 on the vector ALUs (with BF16-rounded weights).
//
// Layout: see policy_tile.h (one wave per 16-agent tile, hidden units as MFMA
// rows, layer 1 -> layer 2 through a per-wave LDS tile).  Small tiles keep the
// tanh work per lane low (16 values per layer) and give a batch many tiles to
// spread over the CUs.

#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "flock_internal.h"
#include "policy_tile.h"

namespace flock {

namespace {

constexpr int kPolBlock = 256;
constexpr int kMaxIn = 257;                    // 256 sectors + speed

// kc: chunks of 32 inputs.
PolLayout carve_pol(char *base, int kc) {
    PolLayout l;
    Carver cv{base, 0};
    l.w1 = cv.take<bf16x8>((size_t)kc * 4 * 64);
    l.w2 = cv.take<bf16x8>(2 * 4 * 64);
    l.w3 = cv.take<bf16x8>(2 * 64);
    l.b1 = cv.take<float>(64);
    l.b2 = cv.take<float>(64);
    l.b3 = cv.take<float>(4);
    l.bytes = align_up(cv.off, 256);
    return l;
}

// Last env e with base[e] <= row.
__device__ __forceinline__ int env_of_row(const int32_t *base, int n_envs, int64_t row) {
    int lo = 0, hi = n_envs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= row) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// What the output layer produces.
enum PolOut {
    kMean = 0,    // actor: the mean action, tanh-squashed and scaled
    kSample = 1,  // actor: mean + sigma * eps and the Gaussian log density of the sample
    kValue = 2,   // critic: the linear first output
};

// Per-launch sampling / value arguments (unused fields are ignored).
struct OutArgs {
    const float2 *eps;  // [n] standard-normal draws (kSample)
    float sig0, sig1;   // exp(log_std) per action dimension
    float logp_c;       // -(log_std0 + log_std1) - log(2 pi)
    float *logp;        // [n] log density of the sample (kSample, may be null)
    float *val;         // [n] critic value (kValue)
    // Tag type filter: when type_want >= 0 only rows of that type (1 chaser,
    // 0 runner; found through the batch tables) are computed and written.
    int type_want;
    const DevEnv *tenvs;
    const int32_t *tbase;
    int tn_envs;
};

// Tile loads a lane keeps in flight while staging obs rows.
constexpr int kStageLoads = 8;

// Rows are agents; obs/act are [n][in_dim] / [n][2] arrays, or, when `envs`
// is non-null, each row's env-owned rows found through the batch tables.
// Layer 1's results reach layer 2's B operand (eight consecutive hidden units
// per lane group) through a per-wave LDS tile [16 agents][72] of BF16.
// kLdsW1: the layer-1 A operand (more than one chunk of 32 inputs) lives in
// LDS, loaded once per block; kStage (batch-wide obs rows): each wave copies
// its tile's 16 consecutive rows, one contiguous block of 16 in_dim floats,
// into LDS as BF16 (zero beyond in_dim) with coalesced 16-byte loads, and the
// MFMA operands are read from there; otherwise every lane loads its own row.

template <bool kLdsW1, int kOut, bool kStage>
__global__ __launch_bounds__(kPolBlock) void k_policy(PolLayout P, int in_dim, int kc,
                                                      float max_turn, float max_dspeed,
                                                      const float *__restrict__ obs, int64_t n,
                                                      float2 *__restrict__ act,
                                                      const DevEnv *__restrict__ envs,
                                                      const int32_t *__restrict__ base,
                                                      int n_envs, OutArgs oa) {
    __shared__ PolConsts s_pc;
    extern __shared__ bf16x8 s_dyn[];
    const int wid = threadIdx.x / 64;
    bf16x8 *s_w1 = s_dyn;  // [kc][4 tiles][64 lanes] when kLdsW1
    __bf16 *s_hid = reinterpret_cast<__bf16 *>(s_dyn + (kLdsW1 ? kc * 256 : 0)) +
                    (size_t)wid * 16 * kHidLd;
    // per-wave obs tiles after the hidden tiles: [16 rows][ld] BF16, ld = 32 kc + 8
    const int ld = 32 * kc + 8;
    __bf16 *s_obs = reinterpret_cast<__bf16 *>(s_dyn + (kLdsW1 ? kc * 256 : 0)) +
                    (size_t)(kPolBlock / 64) * 16 * kHidLd + (size_t)wid * 16 * ld;
    if (kLdsW1)
        for (int i = threadIdx.x; i < kc * 256; i += kPolBlock) s_w1[i] = P.w1[i];
    load_pol_consts(P, &s_pc, threadIdx.x, kPolBlock);
    __syncthreads();

    const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
    bf16x8 w1[4];
    if (!kLdsW1)
#pragma unroll
        for (int t = 0; t < 4; ++t) w1[t] = P.w1[t * 64 + lane];  // kc == 1
    bf16x8 w2[2][4], w3[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int t = 0; t < 4; ++t) w2[c][t] = P.w2[(c * 4 + t) * 64 + lane];
        w3[c] = P.w3[c * 64 + lane];
    }

    const int64_t waves = (int64_t)gridDim.x * (kPolBlock / 64);
    const int64_t tiles = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * (kPolBlock / 64) + wid; tile < tiles;
         tile += waves) {
        const int64_t agent = tile * 16 + col;
        bool valid = agent < n;
        if (oa.type_want >= 0) {
            if (valid) {
                const DevEnv &T = oa.tenvs[env_of_row(oa.tbase, oa.tn_envs, agent)];
                valid = ((agent - T.agent_base) < T.n_chasers ? 1 : 0) == oa.type_want;
            }
            if (!__any(valid)) continue;  // no row of this type in the tile
        }
        const float *orow = obs + agent * in_dim;
        float2 *arow = act + agent;
        if constexpr (kStage) {
            const int64_t row0 = tile * 16;
            const int rows = n - row0 < 16 ? (int)(n - row0) : 16;
            const float *src = obs + row0 * in_dim;
            const int cnt = rows * in_dim, cnt4 = cnt >> 2;
            wave_lds_fence();  // the previous tile's reads come first
            // zero the tile (columns past in_dim must read as 0)
            uint4 *z = reinterpret_cast<uint4 *>(s_obs);
            for (int i = lane; i < 2 * ld; i += 64) z[i] = make_uint4(0u, 0u, 0u, 0u);
            wave_lds_fence();
            int rb = (4 * lane) / in_dim, kb = 4 * lane - rb * in_dim;
            const int dq = 256 / in_dim, dr = 256 - dq * in_dim;
            const float4 *src4 = reinterpret_cast<const float4 *>(src);
            for (int eb = lane; eb < cnt4; eb += 64 * kStageLoads) {
                float4 q[kStageLoads];
#pragma unroll
                for (int u = 0; u < kStageLoads; ++u) {
                    const int e4 = eb + 64 * u;
                    q[u] = src4[e4 < cnt4 ? e4 : cnt4 - 1];  // unconditional: all in flight
                }
#pragma unroll
                for (int u = 0; u < kStageLoads; ++u) {
                    int r = rb, k = kb;
                    rb += dq;
                    kb += dr;
                    if (kb >= in_dim) {
                        kb -= in_dim;
                        ++rb;
                    }
                    if (eb + 64 * u >= cnt4) continue;
                    const float qv[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        s_obs[r * ld + k] = (__bf16)qv[v];
                        if (++k == in_dim) {
                            k = 0;
                            ++r;
                        }
                    }
                }
            }
            for (int e = 4 * cnt4 + lane; e < cnt; e += 64) {
                const int r = e / in_dim;
                s_obs[r * ld + (e - r * in_dim)] = (__bf16)src[e];
            }
            wave_lds_fence();  // this wave's copies before its reads
        }
        if (envs && valid) {
            const DevEnv &E = envs[env_of_row(base, n_envs, agent)];
            const int64_t i = agent - E.agent_base;
            orow = E.obs + i * in_dim;
            arow = reinterpret_cast<float2 *>(E.act) + i;
        }
        // the tile's eight inputs 32 c + 8 g .. + 7 of agent col, as BF16
        auto xb = [&](int c) {
            bf16x8 x;
            const int k0 = 32 * c + 8 * g;
            if constexpr (kStage) {
                x = *reinterpret_cast<const bf16x8 *>(s_obs + col * ld + k0);
            } else if (valid && in_dim % 4 == 0 && k0 + 8 <= in_dim) {
                const float4 *src = reinterpret_cast<const float4 *>(orow + k0);
                const float4 u = src[0], w = src[1];
                x[0] = (__bf16)u.x; x[1] = (__bf16)u.y; x[2] = (__bf16)u.z; x[3] = (__bf16)u.w;
                x[4] = (__bf16)w.x; x[5] = (__bf16)w.y; x[6] = (__bf16)w.z; x[7] = (__bf16)w.w;
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = k0 + j;
                    x[j] = (__bf16)((valid && k < in_dim) ? orow[k] : 0.0f);
                }
            }
            return x;
        };
        auto w1a = [&](int c, int t) { return kLdsW1 ? s_w1[(c * 4 + t) * 64 + lane] : w1[t]; };
        auto w2a = [&](int c, int t) { return w2[c][t]; };
        auto w3a = [&](int c) { return w3[c]; };
        auto hrow = [&](int r) { return s_hid + r * kHidLd; };
        const float2 z = mlp_tile(kc, xb, w1a, w2a, w3a, s_pc, hrow, lane);
        if (g == 0 && valid) {
            if constexpr (kOut == kValue) {
                oa.val[agent] = z.x;
            } else {
                const float2 e = kOut == kSample ? oa.eps[agent] : make_float2(0.0f, 0.0f);
                *arow = pol_output<kOut == kSample>(z, max_turn, max_dspeed, e, oa.sig0,
                                                   oa.sig1, oa.logp_c,
                                                   oa.logp ? oa.logp + agent : nullptr);
            }
        }
    }
}

uint16_t bf16_bits_rne(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float bf16_round(float f) {
    uint32_t u = (uint32_t)bf16_bits_rne(f) << 16;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

}  // namespace

}  // namespace flock

using namespace flock;

struct flock_policy {
    int in_dim, kc;  // kc: chunks of 32 inputs
    int critic;      // 0 actor (two scaled tanh outputs), 1 critic (one linear output)
    float max_turn, max_dspeed;
    PolLayout lay;
    std::vector<char> host;  // staged device image, kept until pol_destroy
};

namespace flock {

namespace {
OutArgs no_filter() {
    OutArgs oa{};
    oa.type_want = -1;
    return oa;
}

template <int kOut>
hipError_t launch_pol(const pol_t *p, const float *obs, int64_t n, float *act, const DevEnv *envs,
                      const int32_t *base, int n_envs, const OutArgs &oa, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int kc = p->kc;
    const int64_t tiles = (n + 15) / 16;
    int64_t blocks = (tiles + 3) / 4;
    if (blocks > 4096) blocks = 4096;
    float2 *a2 = reinterpret_cast<float2 *>(act);
    const bool lds_w1 = kc > 1;
    const size_t w1b = lds_w1 ? (size_t)kc * 256 * sizeof(bf16x8) : 0;
    const size_t hid_b = (size_t)(kPolBlock / 64) * 16 * kHidLd * sizeof(__bf16);
    const size_t tile_b = (size_t)(kPolBlock / 64) * 16 * (32 * kc + 8) * sizeof(__bf16);
    // batch-wide rows whose tiles start 16-byte aligned are staged through LDS
    // (within the 64 KiB of dynamic LDS a launch gets by default)
    const bool stage = obs && !envs && (reinterpret_cast<uintptr_t>(obs) & 15) == 0 &&
                       w1b + hid_b + tile_b <= 65536;
    const size_t lds = w1b + hid_b + (stage ? tile_b : 0);
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kPolBlock), lds, s, p->lay,
                           p->in_dim, kc, p->max_turn, p->max_dspeed, obs, n, a2, envs, base,
                           n_envs, oa);
    };
    if (lds_w1) {
        if (stage) go(k_policy<true, kOut, true>);
        else go(k_policy<true, kOut, false>);
    } else {
        if (stage) go(k_policy<false, kOut, true>);
        else go(k_policy<false, kOut, false>);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t policy_launch(const pol_t *p, const float *obs, int64_t n, float *act, hipStream_t s) {
    return launch_pol<kMean>(p, obs, n, act, nullptr, nullptr, 0, no_filter(), s);
}

hipError_t policy_launch_sample(const pol_t *p, const float *obs, int64_t n, const float *eps,
                                const float log_std[2], float *act, float *logp, hipStream_t s) {
    OutArgs oa = no_filter();
    oa.eps = reinterpret_cast<const float2 *>(eps);
    oa.sig0 = (float)exp((double)log_std[0]);
    oa.sig1 = (float)exp((double)log_std[1]);
    oa.logp_c = (float)(-((double)log_std[0] + (double)log_std[1]) - log(2.0 * M_PI));
    oa.logp = logp;
    return launch_pol<kSample>(p, obs, n, act, nullptr, nullptr, 0, oa, s);
}

hipError_t policy_launch_value(const pol_t *p, const float *obs, int64_t n, float *val,
                               hipStream_t s) {
    OutArgs oa = no_filter();
    oa.val = val;
    return launch_pol<kValue>(p, obs, n, nullptr, nullptr, nullptr, 0, oa, s);
}

hipError_t policy_launch_typed(const pol_t *p, const StepPlan &plan, int table, int type,
                               const float *obs, const float *eps, const float *log_std,
                               float *act, float *logp, hipStream_t s) {
    OutArgs oa{};
    oa.type_want = type;
    oa.tenvs = plan.a.envs[table & 1];
    oa.tbase = plan.a.base;
    oa.tn_envs = plan.n_envs;
    if (!eps) return launch_pol<kMean>(p, obs, plan.G, act, nullptr, nullptr, 0, oa, s);
    oa.eps = reinterpret_cast<const float2 *>(eps);
    oa.sig0 = (float)exp((double)log_std[0]);
    oa.sig1 = (float)exp((double)log_std[1]);
    oa.logp_c = (float)(-((double)log_std[0] + (double)log_std[1]) - log(2.0 * M_PI));
    oa.logp = logp;
    return launch_pol<kSample>(p, obs, plan.G, act, nullptr, nullptr, 0, oa, s);
}

hipError_t policy_launch_envs(const pol_t *p, const StepPlan &plan, int table, hipStream_t s) {
    return launch_pol<kMean>(p, nullptr, plan.G, nullptr, plan.a.envs[table & 1], plan.a.base,
                             plan.n_envs, no_filter(), s);
}

int policy_is_critic(const pol_t *p) { return p->critic; }

const void *policy_weights(const pol_t *p) { return p->lay.w1; }

int policy_in_dim(const pol_t *p) { return p->in_dim; }

PolFuse policy_fuse_args(const pol_t *p) {
    PolFuse f{};
    f.P = p->lay;
    f.in_dim = p->in_dim;
    f.kc = p->kc;
    f.mode = 1;
    f.max_turn = p->max_turn;
    f.max_dspeed = p->max_dspeed;
    return f;
}

void policy_fuse_sampling(PolFuse *f, const float log_std[2], const float *eps, float *logp) {
    f->mode = 2;
    f->eps = reinterpret_cast<const float2 *>(eps);
    f->sig0 = (float)exp((double)log_std[0]);
    f->sig1 = (float)exp((double)log_std[1]);
    f->logp_c = (float)(-((double)log_std[0] + (double)log_std[1]) - log(2.0 * M_PI));
    f->logp = logp;
}

}  // namespace flock

extern "C" {

size_t pol_workspace_bytes(int in_dim, int hidden) {
    if (in_dim < 1 || in_dim > kMaxIn || hidden != kHidden) {
        set_error(ENV_EINVAL, "policy needs 1 <= in_dim <= %d and hidden == 64", kMaxIn);
        return 0;
    }
    return carve_pol(nullptr, (in_dim + 31) / 32).bytes;
}

}  // extern "C"

namespace {

// Shared by the actor (n_out = 2) and the critic (n_out = 1).
int create_net(const float *w, int in_dim, int hidden, int n_out, float max_turn, float max_dspeed,
               void *ws, size_t bytes, void *stream, pol_t **out) {
    if (!w || !ws || !out) return set_error(ENV_EINVAL, "NULL argument to pol_create");
    if (in_dim < 1 || in_dim > kMaxIn || hidden != kHidden)
        return set_error(ENV_EINVAL, "policy needs 1 <= in_dim <= %d and hidden == 64", kMaxIn);
    if (!(max_turn >= 0.0f) || !(max_dspeed >= 0.0f) || !isfinite(max_turn) || !isfinite(max_dspeed))
        return set_error(ENV_EINVAL, "action scales must be finite and >= 0");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return set_error(ENV_EINVAL, "workspace must be 256-byte aligned");
    const int H = kHidden;
    const int kc = (in_dim + 31) / 32;
    const size_t need = carve_pol(nullptr, kc).bytes;
    if (bytes < need)
        return set_error(ENV_ENOMEM, "policy workspace has %zu bytes, needs %zu", bytes, need);
    pol_t *p = new pol_t;
    p->in_dim = in_dim;
    p->kc = kc;
    p->critic = n_out == 1 ? 1 : 0;
    p->max_turn = max_turn;
    p->max_dspeed = max_dspeed;
    p->lay = carve_pol(static_cast<char *>(ws), kc);
    const PolLayout &off = p->lay;
    p->host.assign(need, 0);
    char *hb = p->host.data();
    // host image of the workspace: same offsets from the base as the device arrays
    auto at = [&](const void *dev) {
        return hb + (static_cast<const char *>(dev) - static_cast<const char *>(ws));
    };
    const float *W1 = w;
    const float *b1 = W1 + in_dim * H;
    const float *W2 = b1 + H;
    const float *b2 = W2 + H * H;
    const float *W3 = b2 + H;
    const float *b3 = W3 + H * n_out;
    float *b3d = reinterpret_cast<float *>(at(off.b3));
    for (int o = 0; o < 4; ++o) b3d[o] = o < n_out ? b3[o] : 0.0f;
    // A operands in lane order: lane (g, col) of chunk c, tile t holds
    // W[32 c + 8 g + j][16 t + col] in element j (zero beyond in_dim)
    uint16_t *w1p = reinterpret_cast<uint16_t *>(at(off.w1));
    for (int c = 0; c < kc; ++c)
        for (int t = 0; t < 4; ++t)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    const int k = 32 * c + 8 * (lane / 16) + j, m = 16 * t + lane % 16;
                    const float v = k < in_dim ? W1[k * H + m] : 0.0f;
                    w1p[((c * 4 + t) * 64 + lane) * 8 + j] = bf16_bits_rne(v);
                }
    uint16_t *w2p = reinterpret_cast<uint16_t *>(at(off.w2));
    for (int c = 0; c < 2; ++c)
        for (int t = 0; t < 4; ++t)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    const int k = 32 * c + 8 * (lane / 16) + j, m = 16 * t + lane % 16;
                    w2p[((c * 4 + t) * 64 + lane) * 8 + j] = bf16_bits_rne(W2[k * H + m]);
                }
    // output layer: A[m][k] = W3[k][m] for the n_out real rows m, zero rows after
    uint16_t *w3p = reinterpret_cast<uint16_t *>(at(off.w3));
    for (int c = 0; c < 2; ++c)
        for (int lane = 0; lane < 64; ++lane)
            for (int j = 0; j < 8; ++j) {
                const int k = 32 * c + 8 * (lane / 16) + j, m = lane % 16;
                w3p[(c * 64 + lane) * 8 + j] = bf16_bits_rne(m < n_out ? W3[k * n_out + m] : 0.0f);
            }
    float *b1d = reinterpret_cast<float *>(at(off.b1));
    float *b2d = reinterpret_cast<float *>(at(off.b2));
    for (int h = 0; h < H; ++h) {
        b1d[h] = b1[h];
        b2d[h] = b2[h];
    }
    hipError_t e = hipMemcpyAsync(ws, hb, need, hipMemcpyHostToDevice,
                                  reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        delete p;
        return set_error(ENV_EHIP, "pol_create upload: %s", hipGetErrorString(e));
    }
    *out = p;
    return ENV_OK;
}

}  // namespace

extern "C" {

int pol_create(const float *w, int in_dim, int hidden, float max_turn, float max_dspeed, void *ws,
               size_t bytes, void *stream, pol_t **out) {
    return create_net(w, in_dim, hidden, 2, max_turn, max_dspeed, ws, bytes, stream, out);
}

int pol_create_value(const float *w, int in_dim, int hidden, void *ws, size_t bytes, void *stream,
                     pol_t **out) {
    return create_net(w, in_dim, hidden, 1, 1.0f, 1.0f, ws, bytes, stream, out);
}

void pol_destroy(pol_t *p) { delete p; }

int pol_forward(pol_t *p, const float *obs, int64_t n, float *act, void *stream) {
    if (!p) return set_error(ENV_EINVAL, "policy is NULL");
    if (p->critic) return set_error(ENV_EINVAL, "pol_forward needs an actor (this is a critic)");
    if (n < 0) return set_error(ENV_EINVAL, "n < 0");
    if (n > 0 && (!obs || !act)) return set_error(ENV_EINVAL, "obs/act is NULL");
    hipError_t e = policy_launch(p, obs, n, act, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(ENV_EHIP, "pol_forward: %s", hipGetErrorString(e));
    return ENV_OK;
}

int pol_sample(pol_t *p, const float *obs, int64_t n, const float *log_std, const float *eps,
               float *act, float *logp, void *stream) {
    if (!p || !log_std) return set_error(ENV_EINVAL, "policy or log_std is NULL");
    if (p->critic) return set_error(ENV_EINVAL, "pol_sample needs an actor (this is a critic)");
    if (n < 0) return set_error(ENV_EINVAL, "n < 0");
    if (!isfinite(log_std[0]) || !isfinite(log_std[1]))
        return set_error(ENV_EINVAL, "log_std must be finite");
    if (n > 0 && (!obs || !eps || !act)) return set_error(ENV_EINVAL, "obs/eps/act is NULL");
    hipError_t e = policy_launch_sample(p, obs, n, eps, log_std, act, logp,
                                        reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(ENV_EHIP, "pol_sample: %s", hipGetErrorString(e));
    return ENV_OK;
}

int pol_value(pol_t *p, const float *obs, int64_t n, float *value, void *stream) {
    if (!p) return set_error(ENV_EINVAL, "critic is NULL");
    if (!p->critic) return set_error(ENV_EINVAL, "pol_value needs a critic (pol_create_value)");
    if (n < 0) return set_error(ENV_EINVAL, "n < 0");
    if (n > 0 && (!obs || !value)) return set_error(ENV_EINVAL, "obs/value is NULL");
    hipError_t e = policy_launch_value(p, obs, n, value, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_error(ENV_EHIP, "pol_value: %s", hipGetErrorString(e));
    return ENV_OK;
}

}  // extern "C"
