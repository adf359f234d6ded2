// Internal declarations shared by the kernels (flock_kernels.hip), the C-ABI
// layer (flock_api.cpp), the policy (policy_mfma.hip) and the server
// (server.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "flockenv.h"
#include "policy_tile.h"

namespace flock {

constexpr float kTwoPiF = 6.28318548202514648438f;  // (float)(2 pi)
constexpr int kBlock = 256;                           // threads per block (4 wave64)

// Per-environment descriptor read by every kernel (device memory).
//
// An env keeps its agents in CELL ORDER: record p of the current buffer is
// the p-th agent of the env's last counting sort, and id[p] names that
// agent (its row in agent-order arrays).  Each step reads the current
// buffer and writes the next one in the new cell order (ping-pong), so every
// per-agent access of the step is sequential except the agent-order
// action read and view/reward write.
struct DevEnv {
    float4 *rec_cur, *rec_nxt;   // (x, y, heading, speed), FP32
    int32_t *id_cur, *id_nxt;    // agent index within the env
    double *ret_cur, *ret_nxt;   // FP64 returns
    int32_t *nb, *col;           // agent-order counts (nullptr when not kept)
    // Env-owned agent-order I/O rows, used when a launch gets no batch-wide
    // arrays (serving: rows move between batches as requests come and go).
    float *act;                  // [n][2]
    float *obs;                  // [n][v]
    float *rew;                  // [n]
    int32_t n;                   // agents
    int32_t agent_base;          // first row of this env in batch-wide arrays
    int32_t cell_base;           // first cell of this env in the batch cell space
    // Cell grid: ncx columns of width cw (at least radius / reach), each cut
    // into ncy rows; cell = column * ncy + row.  ncx == 1: all pairs.
    int32_t ncx, ncy;
    int32_t reach;               // stencil half-width in columns (0 when ncx == 1)
    float box;                   // L
    float inv_cx, inv_cy;        // FP32 multipliers: column = floor(x * inv_cx), row likewise
    float cw;                    // column width L / ncx (FP32)
    float marg;                  // widening of the row bounds for FP32 rounding
    float r2;                    // radius^2 (FP32)
    float c2;                    // collide^2 (FP32)
    float inv_radius;            // 1 / radius (FP32)
    float r_nb, r_col;
    float max_turn, max_dspeed, s_min, s_max;
    // View geometry in turns of the bearing from the heading: the arc
    // position is (bearing + fov_half) mod 1, seen iff < fov_t, sector =
    // position * sec_scale.  Full view: fov_half 0, fov_t 1, sec_scale v.
    float fov_half, fov_t, sec_scale;
    int32_t tag;                 // tag environment (runners and chasers)
    int32_t n_chasers;           // tag: agents 0 .. n_chasers-1 are chasers
    float r_catch;               // tag: chaser reward per runner touched
    // Column strips of the strip sort (per plan): strips strip_base ..
    // strip_base + n_strips - 1 of the plan, strip_cols columns each (the
    // last takes the remainder).
    int32_t strip_base, strip_cols, n_strips;
};
static_assert(sizeof(DevEnv) <= 256, "DevEnv grew");

// Device scratch of one counting sort over G agents and C cells.
struct SortArrays {
    int32_t *key;      // [G] new global cell of record p
    int32_t *slot;     // [G] rank of record p within its new cell
    float4 *tmp;       // [G] moved record p (old order)
    float2 *sxy;       // [G] positions in the new cell order (candidates)
    uint8_t *stype;    // [G] tag: 1 for a chaser, in the new cell order
    int32_t *count;    // [C] agents per cell; zero between steps
    int32_t *start;    // [C + 1] exclusive prefix of count
    int32_t *part;     // [scan partials]
    DevEnv *envs[2];   // [E] descriptor tables: [0] as stored, [1] buffers swapped
    int32_t *base;     // [E + 1] agent_base of each env, then G
    // Strip sort (S strips): env of each strip, and the strips' look-back
    // words then the block ticket counter (S + 1 words, zero between steps).
    int32_t *strip_env;  // [S]
    uint32_t *status;    // [S + 1]
    int32_t n_status;    // S + 1 (0 without strips)
};

// The shared policy evaluated inside a step's view sweep, on the view the
// sweep has just produced (still on chip): each agent's next action, written
// to `act` (batch rows [G][2]) or, when `act` is null, to each env's own
// action rows (DevEnv::act).  mode 1: the mean action; mode 2: a Gaussian
// sample round it with the draws `eps` (batch rows) and the log density into
// `logp` (batch rows, may be null).  The actions are bitwise those of
// policy_launch / policy_launch_sample on the same view.
struct PolFuse {
    PolLayout P;
    int in_dim, kc;  // input length (the view row length), chunks of 32 inputs
    int mode;
    float max_turn, max_dspeed;
    float2 *act;
    const float2 *eps;
    float sig0, sig1, logp_c;  // exp(log_std), -(log_std0 + log_std1) - log(2 pi)
    float *logp;
};

// Launch plan of one step over a fixed set of envs.
// Default bound on a strip's look-back wait, in polling rounds.
constexpr int kStripWait = 1 << 14;

struct StepPlan {
    SortArrays a;
    int n_envs;
    int64_t G;    // agents
    int64_t C;    // cells
    int v;        // sectors
    int obs_dim;  // view row length: v, or v + 1 with the speed appended
    int fov;      // any env of the plan has a limited view
    int lanes;    // lanes per agent in the sweep: 1, 4, 16 or 64
    int tag;      // the plan's envs are tag envs (two view channels)
    int scan_blocks;  // 0 -> one scan block per env (every env <= 16384 cells)
    int64_t max_env_cells;  // cells of the plan's largest env
    int env_sort_recs;      // > 0: one block per env does move to scatter (records per thread)
    int strips;             // > 0: the envs' column strips (the strip sort is allowed)
    int strip_now;          // this launch may use the strip sort (every env's records sorted)
    int strip_cells;        // cells of the plan's largest strip
    int strip_cap;          // agents a strip block lists in LDS (more: a second pass)
    // polling rounds a strip waits for the running totals of the strips before
    // it; when they run out it counts the agents before it itself (0: always)
    int strip_wait = kStripWait;
};

// Workspace carving --------------------------------------------------------
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Carves consecutive 256-byte-aligned arrays out of a base pointer; with a
// null base it only accumulates the size (pointers stay null).
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

// Tiles of the two-level scan over C cells, or 0 when every env has few
// enough cells (max_env_cells) for one scan block per env.
int scan_blocks_for(int64_t C, int64_t max_env_cells);
// Records per thread of the per-env fused sort for this plan shape, or 0 when
// the envs are too few to fill the GPU or too large for one block.
int env_sort_recs_for(int n_envs, int64_t max_env_agents, int64_t max_env_cells);
// Carve the sort scratch for G agents, C cells, E envs and S strips.
void carve_sort(Carver &cv, int64_t G, int64_t C, int E, SortArrays *a, int64_t S = 0);
// Strip sort: one block per strip of columns of one env moves the agents of
// its columns and of the two next to them (an agent moves at most one
// column per step), keeps those now in its strip, ranks them by cell in LDS,
// takes its output offset from the strips before it (look-back), and writes
// them in cell order with the strip's cell starts.  Allowed for an env when
// its records are in cell order, its speed limit is at most half a column
// and a strip's cells fit the block's LDS.
constexpr int kStripCells = 8192;
bool strips_allowed(const DevEnv &d);
// Strip width of an env for a plan of G agents in all: columns per strip.
int strip_cols_for(const DevEnv &d, int64_t G);
// Assign strips to the envs' descriptors (in order); returns S and fills
// strip_env with the env index of each strip.
int64_t assign_strips(DevEnv *const *tabs, int n_tabs, int n_envs, int64_t G,
                      std::vector<int32_t> *strip_env);
// Fill the plan's strip_cells / strip_cap from its envs'
// descriptors (after assign_strips) and its strip count.
void plan_strip_launch(StepPlan *p, const DevEnv *envs, int n_envs);

// Launchers (return hipSuccess or the first error) ------------------------
// Zero the cell counts (used once after carving).
hipError_t launch_clear(const StepPlan &p, hipStream_t s);
// Write a one-env plan's descriptor tables (d0 as stored, d1 with the buffers
// swapped) and agent offsets {0, n} into its sort scratch, and zero its counts.
hipError_t launch_bind_one(const StepPlan &p, const DevEnv &d0, const DevEnv &d1, int32_t n,
                           hipStream_t s);
// One step with descriptor table `table` (0 or 1) of the plan.
// do_move = 0 senses the current state without moving (episode start).
// act/obs/reward are batch-wide arrays ([G][2], [G][v], [G]); when NULL the
// kernels use each env's own act/obs/rew rows from its descriptor.
// add_return = 1 adds the reward to the FP64 returns.
// Whether a step of this plan can run the policy in its view sweep (PolFuse):
// flock plans whose sweep uses one or four lanes per agent (blocks of 256 or
// 64 agents, over which the network's weights are staged once).
bool plan_fuses_policy(const StepPlan &p);
// pf (not null): the policy runs in the sweep (see PolFuse); only for plans
// with plan_fuses_policy (hipErrorInvalidValue otherwise).
// act_copy (not null, batch rows [G][2]): the move also writes each applied
// action (as read, before its clamp) there.
hipError_t launch_step(const StepPlan &p, int table, int do_move, const float *act, float *obs,
                       float *reward, int add_return, hipStream_t s,
                       hipEvent_t *phase_events = nullptr, const PolFuse *pf = nullptr,
                       float *act_copy = nullptr);
// The step's phases, in order.  Data they share: move writes tmp/key/slot and
// the counts and reads the current records; scan turns counts into starts;
// scatter writes the next records, sxy and stype; sweep reads those and the
// starts.
enum StepPhase { kPhaseMove = 0, kPhaseScan = 1, kPhaseScatter = 2, kPhaseSweep = 3 };
hipError_t launch_phase(const StepPlan &p, int table, StepPhase phase, int do_move,
                        const float *act, float *obs, float *reward, int add_return,
                        hipStream_t s, const PolFuse *pf = nullptr, float *act_copy = nullptr);
// Load an agent-order state into buffer `rec`/`id` (identity order).
hipError_t launch_load_state(const float *x, const float *y, const float *th, const float *sp,
                             float4 *rec, int32_t *id, int n, hipStream_t s);
// Agent-order state / returns out of a cell-order buffer.
hipError_t launch_store_state(const float4 *rec, const int32_t *id, float *x, float *y,
                              float *th, float *sp, int n, hipStream_t s);
hipError_t launch_store_returns(const double *ret, const int32_t *id, double *out, int n,
                                hipStream_t s);
// Agent-order returns `in` into a cell-order buffer: ret[p] = in[id[p]].
hipError_t launch_load_returns(const double *in, const int32_t *id, double *ret, int n,
                               hipStream_t s);
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s);
hipError_t launch_copy_i32(const int32_t *src, int32_t *dst, int64_t n, hipStream_t s);

// Env internals used by the batch and serving layers (flock_api.cpp) -------
int validate_params(const env_params_t *p);     // ENV_OK or ENV_EINVAL (+ message)
bool full_view(const env_params_t &p);          // fov 0 or 2 pi: the whole circle
int obs_dim_of(const env_params_t &p);          // view row length: sectors (+ 1 for speed)
// Expected candidate tests per agent of an env (uniform density over its grid).
double env_candidates_per_agent(const env_t *env);
// Sweep lanes per agent for a mean of `cand` candidate tests per agent, v
// sectors, `agents` agents in the launch.
int auto_lanes(double cand, int v, int64_t agents);
// Descriptor with agent_base = cell_base = 0, oriented so that rec_cur is
// the env's current buffer (flip = 1 swaps cur and nxt).
DevEnv env_descriptor(const env_t *env, int flip);
int64_t env_cell_count(const env_t *env);       // cells of this env's grid
int64_t cell_count_for(const env_params_t &p);  // cells an env of these params uses
int64_t column_count_for(const env_params_t &p); // grid columns of such an env
const env_params_t &env_params(const env_t *env);
int env_parity(const env_t *env);
void env_advance(env_t *env, int steps);        // record `steps` stepped elsewhere
bool env_sorted(const env_t *env);              // records in cell order (strip sort allowed)
// Copy a host state into the env (async on s; host arrays must outlive the copy).
int env_load_host_state(env_t *env, const float *x, const float *y, const float *th,
                        const float *s_, hipStream_t s);
// Device FP64 returns of the env in agent order, into `out` (device [n]).
int env_returns_to(env_t *env, double *out, hipStream_t s);
// Bytes of the batch sort scratch for G agents, C cells, E envs, S strips.
size_t sort_scratch_bytes(int64_t G, int64_t C, int E, int64_t S = 0);

// Policy network (policy_mfma.hip) ---------------------------------------------
// act[n][2] = policy(obs[n][in_dim]) on `s`.
hipError_t policy_launch(const pol_t *pol, const float *obs, int64_t n, float *act, hipStream_t s);
// Over every row of a batch plan, reading obs and writing act through each
// env's own rows (DevEnv::obs / DevEnv::act) of descriptor table `table`.
hipError_t policy_launch_envs(const pol_t *pol, const StepPlan &plan, int table, hipStream_t s);
int policy_in_dim(const pol_t *pol);
// The actor's arguments for a fused step (mode 1, mean action, act = null).
PolFuse policy_fuse_args(const pol_t *pol);
// pf with Gaussian sampling (mode 2) as policy_launch_sample.
void policy_fuse_sampling(PolFuse *pf, const float log_std[2], const float *eps, float *logp);
int policy_is_critic(const pol_t *pol);
// Device address of the policy's weights (identifies what a captured graph reads).
const void *policy_weights(const pol_t *pol);
// act = mean + exp(log_std) * eps (eps [n][2]), logp [n] (may be null).
hipError_t policy_launch_sample(const pol_t *pol, const float *obs, int64_t n, const float *eps,
                                const float log_std[2], float *act, float *logp, hipStream_t s);
// Tag: rows of one type (1 chasers, 0 runners) of a batch plan; mean
// action when eps is null, else sampled as policy_launch_sample.
hipError_t policy_launch_typed(const pol_t *pol, const StepPlan &plan, int table, int type,
                               const float *obs, const float *eps, const float *log_std,
                               float *act, float *logp, hipStream_t s);
// value [n] = critic(obs).
hipError_t policy_launch_value(const pol_t *pol, const float *obs, int64_t n, float *value,
                               hipStream_t s);

// Error channel shared by every C entry point (flock_api.cpp): records a
// thread-local message for env_last_error() and returns `code`.
int set_error(int code, const char *fmt, ...);

}  // namespace flock
