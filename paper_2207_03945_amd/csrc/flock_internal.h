// Internal declarations shared by the kernels (flock_kernels.hip) and the
// C-ABI layer (flock_api.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "flockenv.h"

namespace flock {

constexpr float kTwoPiF = 6.28318548202514648438f;  // (float)(2 pi)
constexpr int kBlock = 256;                           // threads per block (4 wave64)

// Per-environment descriptor read by every kernel (device memory).
struct DevEnv {
    float *x, *y, *th, *s;  // state, FP32 [n]
    double *ret;            // FP64 returns [n]
    int32_t *nb, *col;      // counts [n] (nullptr when not kept)
    // Env-owned I/O rows, used when a launch gets no batch-wide arrays
    // (serving: rows move between batches as requests come and go).
    float *act;             // [n][2]
    float *obs;             // [n][v]
    float *rew;             // [n]
    int32_t n;              // agents
    int32_t agent_base;     // first row of this env in batch-wide arrays
    int32_t cell_base;      // first cell of this env in the batch cell space
    int32_t ncell;          // cells per side (1 = all pairs)
    int32_t reach;          // stencil half-width in cells (0 when ncell == 1)
    float box;              // L
    float inv_cell;         // FP32 multiplier: cell = floor(x * inv_cell)
    float r2;               // radius^2 (FP32)
    float c2;               // collide^2 (FP32)
    float radius;
    float r_nb, r_col;
    float max_turn, max_dspeed, s_min, s_max;
    float sec_scale;        // FP32(v / 2pi)
};
static_assert(sizeof(DevEnv) <= 160, "DevEnv grew");

// Device arrays of one cell-list sort over G agents and C cells.
struct SortArrays {
    int32_t *key;     // [G] global cell of each agent (row order)
    int32_t *slot;    // [G] rank within its cell (arrival order of the atomic)
    float4 *tmp;      // [G] (x', y', cos th', sin th') in row order
    float2 *sxy;      // [G] positions in cell order
    float2 *scs;      // [G] (cos, sin) of heading in cell order
    int32_t *perm;    // [G] row of the agent at each cell-order position
    int32_t *count;   // [C] agents per cell; zero between steps
    int32_t *start;   // [C + 1] exclusive prefix of count
    int32_t *part;    // [scan partials]
    uint32_t *ticket; // [1] scan completion counter; zero between steps
    DevEnv *envs;     // [E] descriptors
    int32_t *base;    // [E + 1] agent_base of each env, then G
};

// Launch plan of one step over a fixed set of envs.
struct StepPlan {
    SortArrays a;
    int n_envs;
    int64_t G;    // agents
    int64_t C;    // cells
    int v;        // sectors
    int flags;
    int scan_blocks;  // 0 -> single-block scan
};

// Workspace carving --------------------------------------------------------
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Carver {
    char *base;
    size_t off;
    template <typename T>
    T *take(size_t count) {
        off = align_up(off, 256);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Number of scan partial blocks for C cells (0 = one block does everything).
int scan_blocks_for(int64_t C);
// Carve the sort arrays for G agents, C cells and E envs.
void carve_sort(Carver &cv, int64_t G, int64_t C, int E, SortArrays *a);

// Launchers (return hipSuccess or the first error) ------------------------
// Zero count and ticket (used once after carving).
hipError_t launch_clear(const StepPlan &p, hipStream_t s);
// Full step; do_move = 0 senses the current state without moving (reset).
// act/obs/reward are batch-wide arrays ([G][2], [G][v], [G]); when NULL the
// kernels use each env's own act/obs/rew rows from its descriptor.
hipError_t launch_step(const StepPlan &p, int do_move, const float *act, float *obs,
                       float *reward, int add_return, hipStream_t s,
                       hipEvent_t *phase_events = nullptr);
// Copy state in or out of one env.
hipError_t launch_copy_state(const float *sx, const float *sy, const float *sth,
                             const float *ss, float *dx, float *dy, float *dth, float *ds,
                             int n, hipStream_t s);
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s);
hipError_t launch_copy_i32(const int32_t *src, int32_t *dst, int64_t n, hipStream_t s);
hipError_t launch_copy_f64(const double *src, double *dst, int64_t n, hipStream_t s);

// Policy network (policy_mfma.hip) ---------------------------------------------
// act[n][2] = policy(obs[n][in_dim]) on `s`.
hipError_t policy_launch(const pol_t *pol, const float *obs, int64_t n, float *act, hipStream_t s);
// Over every row of a batch plan, reading obs and writing act through each
// env's own rows (DevEnv::obs / DevEnv::act).
hipError_t policy_launch_envs(const pol_t *pol, const StepPlan &plan, hipStream_t s);
int policy_in_dim(const pol_t *pol);

// Env internals used by the serving loop (flock_api.cpp) ---------------------
int validate_params(const env_params_t *p);     // ENV_OK or ENV_EINVAL (+ message)
DevEnv env_descriptor(const env_t *env);        // agent_base / cell_base are 0
int64_t env_cell_count(const env_t *env);       // cells of this env's grid
const env_params_t &env_params(const env_t *env);
// Copy a host state into the env (async on s; host arrays must outlive the copy).
int env_load_host_state(env_t *env, const float *x, const float *y, const float *th,
                        const float *s_, hipStream_t s);
// Bytes of the batch sort scratch for G agents, C cells, E envs.
size_t sort_scratch_bytes(int64_t G, int64_t C, int E);

// Error channel shared by every C entry point (flock_api.cpp): records a
// thread-local message for env_last_error() and returns `code`.
int set_error(int code, const char *fmt, ...);

}  // namespace flock
