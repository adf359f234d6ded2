/*
 * flockenv.h -- C ABI of the MI355X flock-environment step library.
 *
 * The environment is the "flock" multi-agent environment of Langham-Lopez,
 * Schmon and Cannon, "High Performance Simulation for Scalable Multi-Agent
 * Reinforcement Learning" (arXiv:2207.03945):
 *   - Sec. 2.1: discrete time; every interaction updates all agents
 *     simultaneously.
 *   - Sec. 2.2: environment and learner share device memory directly, with no
 *     copy through the host.
 *   - Sec. 4: each agent's view is v sectors of its field of view, each
 *     holding the distance to the nearest other agent at that bearing.
 *   - Sec. 4.1: actions rotate the heading (at most theta_max) and change the
 *     speed (clamped to [s_min, s_max]); reward Eq. (1) sums a contribution
 *     over all agents closer than the vision range d_v, with a penalty for a
 *     collision (Fig. 4); each update first applies the actions, then updates
 *     the view and reward over all pairs in spatial proximity.
 *   - Sec. 4.3 and 5: one policy network shared by all agents, two hidden
 *     layers of 64 units.
 *
 * Conventions for every call below:
 *   - Every pointer named in a "device" argument is device memory of the
 *     current HIP device (for example a PyTorch CUDA tensor's data_ptr()).
 *     "host" pointers are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously on it; the caller synchronises.
 *   - The library never allocates device memory.  All device memory is a
 *     caller-owned workspace whose size the *_workspace_bytes call reports;
 *     the workspace must stay alive, untouched by the caller, until the
 *     object bound to it is destroyed.
 *   - Return value: ENV_OK (0) on success, a negative ENV_E* code on error.
 *     On error nothing is enqueued and no state changes; env_last_error()
 *     returns a message for the calling thread.
 *   - An object is used from one host thread and one stream at a time.
 *
 * State layout (structure of arrays, FP32, agent order): x[n], y[n] in
 * [0, box), heading th[n] in [0, 2pi), speed s[n] in [s_min, s_max].
 * Actions act[n][2]: column 0 = turn (rad), column 1 = speed change (the
 * speed itself for tag envs).  View obs[n][d] (agent-major): d = v (2v for
 * tag envs), + 1 with ENV_FLAG_SPEED_OBS; 1 - d_min/radius per sector, 0
 * when empty, then the agent's speed.  Reward reward[n] = r_nb *
 * n_neighbours + r_col * n_collisions (tag envs: see env_params_t).
 */
#ifndef FLOCKENV_H
#define FLOCKENV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#pragma GCC visibility push(default)
#endif

enum {
    ENV_OK = 0,
    ENV_EINVAL = -1,   /* bad argument or parameter                      */
    ENV_ENOMEM = -2,   /* workspace (or arena / budget) too small         */
    ENV_ESTATE = -3,   /* call out of order (e.g. step before reset)     */
    ENV_EHIP = -4,     /* HIP runtime error (message names the call)     */
    ENV_EAGAIN = -5,   /* serving: request queued, no slot or memory yet */
    ENV_ENOTFOUND = -6 /* serving: unknown request id                    */
};

/* flags */
#define ENV_FLAG_COUNTS 1    /* keep per-agent neighbour / collision counts   */
#define ENV_FLAG_SPEED_OBS 2 /* append the agent's speed to its view row      */
#define ENV_FLAG_TAG 4       /* tag environment: runners and chasers          */

/*
 * Environment parameters (Sec. 4.1).  Requirements, else ENV_EINVAL:
 * 0 <= n_agents <= 2^26; box finite and > 0; 0 < radius < box/2 (so the
 * nearest periodic image is unique within the vision range);
 * 0 <= collide <= radius; 1 <= sectors <= 256; max_turn, max_dspeed >= 0;
 * 0 <= s_min <= s_max; all finite; cell_reach in {0, 1, 2} (0 = default 1):
 * grid columns are at least radius/cell_reach wide, so 2 cell_reach + 1 of
 * them cover the vision disc.  Boxes narrower than three columns use a
 * single cell and compare all pairs; the result does not depend on this.
 * fov: field of view in radians, in [0, 2pi] (FP32 2pi); 0 and 2pi mean
 * all round (Sec. 5 uses about 250 degrees).  With a full view sector 0 starts at the heading;
 * with a limited view the v sectors split the arc [-fov/2, fov/2) round the
 * heading from its right edge, counter-clockwise.  Agents outside the arc
 * are not seen but still count in the reward (Eq. (1)).  A coincident
 * agent is taken to lie on the heading.
 *
 * Tag (ENV_FLAG_TAG, Sec. 4.2): agents 0 .. n_chasers-1 are chasers, the
 * rest runners (0 <= n_chasers <= n_agents).  The second action component
 * is the speed itself, clamped to [0, s_max] (max_dspeed and s_min are not
 * used).  The view has two channels of v sectors, runners then chasers
 * (row length 2v, + 1 with ENV_FLAG_SPEED_OBS).  A touch is a pair of
 * different types closer than `collide`.  Counts: n_nb = runners within
 * `radius`, n_col = touches.  Reward: runner r_nb n_nb + r_col n_col,
 * chaser r_catch n_col.  Tag and flock envs do not mix in a batch.
 */
typedef struct env_params {
    int32_t n_agents;
    float box;         /* side L of the periodic square box              */
    float radius;      /* vision range d_v (Eq. (1))                     */
    float collide;     /* collision distance 2 d_r (Fig. 4)              */
    int32_t sectors;   /* v (Sec. 4)                                     */
    float r_nb;        /* reward per neighbour within radius             */
    float r_col;       /* reward per collision (negative = penalty)      */
    float max_turn;    /* theta_max (Sec. 4.1)                           */
    float max_dspeed;  /* a_max (Sec. 4.1)                               */
    float s_min;       /* speed clamp (Sec. 4.1)                         */
    float s_max;
    int32_t cell_reach;
    int32_t flags;     /* ENV_FLAG_*                                     */
    float fov;         /* field of view (radians), 0 = full              */
    int32_t n_chasers; /* tag: agents 0 .. n_chasers-1 are chasers       */
    float r_catch;     /* tag: chaser reward per runner it touches       */
} env_params_t;

typedef struct flock_env env_t;
typedef struct flock_batch env_batch_t;
typedef struct flock_policy pol_t;
typedef struct flock_server srv_t;

/* Thread-local message describing the last error ("" if none). */
const char *env_last_error(void);

/* ------------------------------------------------------------------ env */

/* Device bytes one environment needs (state, FP64 returns, counts and the
 * cell-list scratch of its own step).  0 if the parameters are invalid. */
size_t env_workspace_bytes(const env_params_t *p);

/* Bind an environment to `workspace` (device, >= env_workspace_bytes(p)
 * bytes, 256-byte aligned).  Makes no HIP call.  *out receives a handle the
 * caller releases with env_destroy.  ENV_EINVAL (bad params, NULL or
 * misaligned pointer), ENV_ENOMEM (bytes too small). */
int env_create(const env_params_t *p, void *workspace, size_t bytes, env_t **out);

/* Release the handle (not the workspace).  NULL is ignored. */
void env_destroy(env_t *env);

/* Effective cell grid: ncx columns of width cell_w (at least radius /
 * reach; 1 column = all pairs), each cut into ncy rows of height cell_h
 * (ncy = 4 ncx, or 1 for all pairs); the sweep visits 2 reach + 1 columns
 * and, in each, only the rows that can hold a point within the vision
 * radius.  Any output pointer may be NULL.  ENV_EINVAL for a NULL env. */
int env_geometry(const env_t *env, int32_t *ncx, int32_t *ncy, int32_t *reach, float *cell_w,
                 float *cell_h);

/* Lanes of the neighbour sweep that share one agent's candidates (a lane
 * group inside a wavefront): 1, 4, 16 or 64, or 0 to choose from the
 * expected candidates per agent (about n (2 reach + 1) cell_w (2 radius +
 * cell_h) / box^2).
 * Results do not depend on it; sparse neighbourhoods favour 1, dense ones
 * (hundreds of candidates per agent) larger groups, and so do steps with few
 * agents in all (the automatic choice takes 64 up to 8,192 agents and 16 up
 * to 16,384, where wider groups keep more compute units busy).  The
 * automatic choice assumes uniform density; clustered states may do better
 * with a larger group.  ENV_EINVAL for other values. */
int env_set_sweep_lanes(env_t *env, int lanes);

/* Copy a state in (device x, y, th, s, each [n] FP32).  Values must already
 * lie in their ranges (positions in [0, box), heading in [0, 2pi)); they are
 * not checked.  Enqueued on `stream`. */
int env_set_state(env_t *env, const float *x, const float *y, const float *th,
                  const float *s, void *stream);

/* Copy the current state out (device x, y, th, s, each [n] FP32). */
int env_get_state(env_t *env, float *x, float *y, float *th, float *s, void *stream);

/* Start an episode from the current state: zero the FP64 returns and compute
 * the initial view obs (device [n][d] FP32) without moving.  Requires a
 * prior env_set_state, else ENV_ESTATE. */
int env_reset(env_t *env, float *obs, void *stream);

/* One step (Sec. 4.1 order): apply act (device [n][2]) to every agent, move,
 * then write the view obs (device [n][d]) and reward (device [n]) of the new
 * positions, and add the reward to the FP64 returns.  ENV_ESTATE before
 * env_reset. */
int env_step(env_t *env, const float *act, float *obs, float *reward, void *stream);

/* Last step's per-agent neighbour / collision counts (device int32 [n]);
 * requires ENV_FLAG_COUNTS, else ENV_ESTATE. */
int env_get_counts(env_t *env, int32_t *n_nb, int32_t *n_col, void *stream);

/* Per-agent undiscounted returns since env_reset (device FP64 [n]). */
int env_get_returns(env_t *env, double *ret, void *stream);

/* Overwrite the per-agent FP64 returns (device [n], agent order), for
 * resuming an episode from a checkpoint: env_set_state, env_reset (which
 * zeroes the returns), then env_set_returns with the saved values.  The
 * returns are the undiscounted sums of Eq. (1)'s rewards that env_step keeps
 * adding to.  ENV_ESTATE before env_reset. */
int env_set_returns(env_t *env, const double *ret, void *stream);

/* For callers that cannot allocate device memory or hand the library a
 * scratch workspace at step time: code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc.  The same step as env_step (bitwise
 * the same results), but its sort scratch comes from a static device array
 * of env_static_scratch_bytes() bytes (32 MiB) per GPU, held until the
 * process ends; the call allocates nothing.  The env still owns its state
 * in its workspace; act, obs and reward are as for env_step.  ENV_ENOMEM
 * (before anything is enqueued) when the step needs more scratch than the
 * array holds: about 33 bytes per agent plus 8 per grid cell, so roughly
 * 800,000 agents at the default grid.  Every call on one GPU uses that GPU's
 * array: calls that overlap on one GPU (two streams, or two threads) race and
 * must be serialised by the caller.  The env's device must be current. */
size_t env_static_scratch_bytes(void);
int env_step_static(env_t *env, const float *act, float *obs, float *reward, void *stream);

/* ---------------------------------------------------------------- batch */

/* Several environments (possibly of different sizes, boxes and views;
 * equal `sectors` and ENV_FLAG_SPEED_OBS) stepped together by one sequence
 * of launches: Sec. 2.1 has the engine update all entities of a timestep in
 * parallel on the GPU, and Sec. 5 trains many independent environments at
 * once; a batch is such a set sharing one launch.  Agents of env k
 * occupy rows [off[k], off[k+1]) of the batch-wide act/obs/reward arrays,
 * with off[k] = sum of n_agents of envs 0..k-1 (see env_batch_offsets).
 * Results are bitwise identical to stepping each env with env_step. */
size_t env_batch_workspace_bytes(env_t *const *envs, int n_envs);

/* (The workspace also holds G next actions for env_step_policy.)
 * `ws` is device memory of >= env_batch_workspace_bytes bytes; the batch
 * borrows the envs, which must outlive it.  Every env must have had
 * env_reset.  ENV_EINVAL (n_envs < 1, NULL env, mixed sectors or flags),
 * ENV_ENOMEM. */
int env_batch_create(env_t *const *envs, int n_envs, void *ws, size_t bytes,
                     env_batch_t **out);
void env_batch_destroy(env_batch_t *b);

/* As env_set_sweep_lanes, for the batched step (Sec. 4: the sweep that
 * builds every agent's view; 0 = chosen from the
 * agent-weighted mean of the envs' expected candidates).  Drops captured
 * graphs when the choice changes. */
int env_batch_set_sweep_lanes(env_batch_t *b, int lanes);
/* *lanes receives the lanes per agent the batched sweep uses now. */
int env_batch_get_sweep_lanes(const env_batch_t *b, int32_t *lanes);

/* Policy fusion for env_step_policy and env_rollout (Sec. 4.3: one policy
 * shared by all agents acting on their own views), off by default.  When on,
 * and the batch's sweep uses one or four lanes per agent, the policy runs
 * inside the step's view sweep on the views it has just produced (still in
 * LDS), so no separate policy launch reads them back: env_rollout evaluates
 * only its first action separately; env_step_policy keeps the next step's
 * actions in the batch workspace and applies them on the next call with the
 * same pol and obs pointer when no env of the batch changed in between (any
 * other stepping call, env_set_state or env_reset), so obs must not be
 * written between such calls.  Results are bitwise the same either way.  Off
 * by default because on MI355X the fused step is slower: the network's tanh
 * work is vector-ALU bound and its registers and LDS lower the occupancy of
 * the issue-bound sweep.  ENV_EINVAL for a NULL batch. */
int env_batch_set_policy_fusion(env_batch_t *b, int on);

/* Bound on the wait of the batch's strip sort (polling rounds; default
 * 16384).  The sort cuts each env's grid columns into strips, one block each,
 * and a strip takes its first output row from the running totals of the
 * strips before it; a strip whose wait runs out counts the agents before it
 * itself.  Results are the same for every value: 0 makes every strip count
 * (the fallback, for tests).  Drops captured graphs when the value changes.
 * ENV_EINVAL for a NULL batch or polls < 0. */
int env_batch_set_strip_wait(env_batch_t *b, int polls);

/* off[n_envs + 1] (host) receives the row offsets described above
 * (the per-agent arrays of Sec. 4.1 laid end to end).  ENV_EINVAL for a
 * NULL batch or off. */
int env_batch_offsets(const env_batch_t *b, int64_t *off);

/* One step of every env in the batch (Sec. 4.1, as env_step; Sec. 2.1: all
 * agents of all envs in one timestep).  act: device [G][2], obs: device
 * [G][d] (d as for env_step), reward: device [G], G = off[n_envs]; all
 * caller-owned, agent order.  ENV_EINVAL for NULL arguments, ENV_EHIP when
 * a launch fails. */
int env_step_batched(env_batch_t *b, const float *act, float *obs, float *reward,
                     void *stream);

/* k_steps consecutive batched steps (Sec. 2.1's discrete timesteps, each as
 * env_step_batched) replayed from a captured HIP graph.
 * act: device [k_steps][G][2] (step-major), obs: device [G][d] (final view),
 * reward: device [k_steps][G].  The graph is captured on the first call and
 * re-captured when any argument changes. */
int env_batch_run(env_batch_t *b, int k_steps, const float *act, float *obs,
                  float *reward, void *stream);

/* Capture (or re-capture) the graph env_batch_run would replay for these
 * arguments, without launching it.  Same arguments and errors. */
int env_batch_capture(env_batch_t *b, int k_steps, const float *act, float *obs,
                      float *reward, void *stream);

/* One env_step_batched whose four phases are bracketed by HIP events on
 * `stream`: phase_ms[0] move + cell count, [1] scan, [2] scatter, [3]
 * neighbour sweep (milliseconds).  Where one kernel sorts (each env of a
 * batch of many small envs, or each strip of grid columns once the batch is
 * in cell order) it moves, counts, scans and scatters together: phase_ms[0]
 * is then that kernel and [1], [2] are 0.  Synchronises the stream.  For
 * profiling; results are the same as env_step_batched. */
int env_step_batched_timed(env_batch_t *b, const float *act, float *obs, float *reward,
                           void *stream, float *phase_ms);

/* --------------------------------------------------------------- policy */

/* Shared policy network of Sec. 4.3/5: in -> hidden -> hidden -> 2, tanh on
 * every layer, output scaled by (max_turn, max_dspeed).  in lies in
 * [1, 257] and, where the policy drives envs, equals their view row length
 * d (sectors, + 1 with ENV_FLAG_SPEED_OBS); hidden = 64.  Sec. 5's flock
 * network reads d = 129 (128 sectors and the speed). */
size_t pol_workspace_bytes(int in_dim, int hidden);

/* w_host: FP32 host array W1[in][hidden], b1[hidden], W2[hidden][hidden],
 * b2[hidden], W3[hidden][2], b3[2] (row-major, fan_in x fan_out).  Weights
 * are rounded once to BF16 (round to nearest even) into `ws`; biases stay
 * FP32.  Enqueued on `stream` (the copy is complete when the stream is). */
int pol_create(const float *w_host, int in_dim, int hidden, float max_turn,
               float max_dspeed, void *ws, size_t bytes, void *stream, pol_t **out);
void pol_destroy(pol_t *pol);

/* act[n][2] = policy(obs[n][in]) (device), BF16 MFMA, FP32 accumulate. */
int pol_forward(pol_t *pol, const float *obs, int64_t n, float *act, void *stream);

/* Critic network of Sec. 5 (two hidden layers of 64, tanh): in -> hidden ->
 * hidden -> 1, linear output.  w_host: W1[in][hidden], b1[hidden],
 * W2[hidden][hidden], b2[hidden], W3[hidden][1], b3[1]; same precision and
 * workspace size (pol_workspace_bytes) as the actor.  The handle works only
 * with pol_value; pol_destroy releases it. */
int pol_create_value(const float *w_host, int in_dim, int hidden, void *ws, size_t bytes,
                     void *stream, pol_t **out);

/* value[n] = critic(obs[n][in]) (device FP32).  ENV_EINVAL for an actor. */
int pol_value(pol_t *critic, const float *obs, int64_t n, float *value, void *stream);

/* PPO's Gaussian action sampling round the actor's mean (Sec. 4.3, Fig. 5):
 * act[i] = mean_i + exp(log_std) * eps[i] (eps: device [n][2] standard
 * normal draws, supplied by the caller), and, when logp is not NULL,
 * logp[i] = -(eps_i0^2 + eps_i1^2)/2 - log_std_0 - log_std_1 - log(2 pi),
 * the log density of the sample.  log_std: host float[2].  The environment
 * clamps the sampled action to its range when it applies it. */
int pol_sample(pol_t *pol, const float *obs, int64_t n, const float *log_std, const float *eps,
               float *act, float *logp, void *stream);

/* Experience collection (Sec. 4.3, Fig. 5; Sec. 5: t = 128 updates per
 * training step): `steps` closed-loop batched steps whose views, actions,
 * log densities and rewards are written straight into the caller's rollout
 * buffers (device, rows in batch order, G = off[n_envs], d as for env_step):
 *   obs    [steps + 1][G][d]  block 0 holds the current view on entry
 *                             (from env_reset or the last step); block
 *                             k + 1 receives the view after step k
 *   act    [steps][G][2]      actions taken (sampled, before the clamp)
 *   logp   [steps][G]         log density of each sample (NULL: not kept)
 *   reward [steps][G]
 * eps (device [steps][G][2] standard normals) and log_std (host float[2])
 * select Gaussian sampling as pol_sample; eps = NULL takes the mean action
 * (then logp must be NULL).  FP64 returns accumulate as for env_step.  The
 * launches of all steps are captured once into a HIP graph and replayed
 * (re-captured when an argument changes); `stream` must not be the null
 * stream.  Results equal `steps` rounds of pol_sample (or pol_forward) and
 * env_step_batched, bitwise (also with env_batch_set_policy_fusion on, when
 * only the first action comes from a separate policy evaluation and each
 * step's view sweep evaluates and samples the next one). */
int env_rollout(env_batch_t *b, pol_t *pol, int steps, const float *log_std, const float *eps,
                float *obs, float *act, float *logp, float *reward, void *stream);

/* Tag rollout (Sec. 4.2, 4.3: runners and chasers train independent
 * policies): as env_rollout, with each row's action from the policy of its
 * agent's type.  log_std: host float[4], the runner's two values then the
 * chaser's.  ENV_EINVAL unless the batch holds tag envs. */
int env_rollout_tag(env_batch_t *b, pol_t *runner, pol_t *chaser, int steps,
                    const float *log_std, const float *eps, float *obs, float *act, float *logp,
                    float *reward, void *stream);

/* Tag closed-loop step: act = runner or chaser policy (mean action) of each
 * row's obs by its type, then one batched step, as env_step_policy. */
int env_step_policy_tag(env_batch_t *b, pol_t *runner, pol_t *chaser, float *act, float *obs,
                        float *reward, void *stream);

/* PPO's truncated advantage estimator over a rollout (Sec. 4.3, Sec. 5), per
 * agent: delta_t = r_t + gamma V_{t+1} - V_t, A_t = delta_t + gamma lambda
 * A_{t+1} with A_steps = 0, and value targets R_t = A_t + V_t.
 * reward [steps][n], value [steps + 1][n] (row `steps` is the bootstrap
 * value of the state after the last step), adv and ret [steps][n]; device
 * FP32, evaluated in FP64 and rounded once.  gamma, lambda in [0, 1]. */
int rl_gae(int steps, int64_t n, float gamma, float lambda, const float *reward,
           const float *value, float *adv, float *ret, void *stream);

/* Closed-loop batched step (Sec. 4.3: one policy shared by all agents, each
 * acting on its own view): act = policy(obs) for every agent, then one
 * batched step with those actions.  obs (device [G][d]) is read as the
 * current view and overwritten by the new one; act (device [G][2]) receives
 * the actions taken; reward (device [G]).
 * The actions are bitwise those of pol_forward on the same views.  With
 * env_batch_set_policy_fusion on (and a sweep of one or four lanes per
 * agent), see there. */
int env_step_policy(env_batch_t *b, pol_t *pol, float *act, float *obs, float *reward,
                    void *stream);

/* ---------------------------------------------------- graph interaction */

/* One step of the opinion-dynamics model of Sec. 2.1 (the engine's
 * interaction over graph edges): for every node i and each incoming edge e
 * = (i, j) in CSR order, when |op_in[i] - op_in[j]| < threshold (FP32),
 * new_i <- (1 - strength w_e) new_i + strength w_e op_in[j], starting from
 * new_i = op_in[i]; then op_out[i] = new_i (the self interaction).  Every
 * test reads the step's input opinions.
 *   row_ptr  device int64 [n + 1]: edges of node i are row_ptr[i] ..
 *            row_ptr[i + 1] - 1 (ranges are clamped to [0, n_edges])
 *   col      device int32 [n_edges]: j of each edge (j outside [0, n) is
 *            skipped)
 *   weight   device FP32 [n_edges]
 *   op_in, op_out  device FP32 [n], distinct
 * Updates run in FP64, rounded once to FP32.  lanes: lanes per node (1, 4,
 * 16, 64; 0 = from the mean degree).  With lanes = 1 each node applies its
 * edges one by one in the stated order; with more, chunks of the row are
 * composed as affine maps (the same map up to FP64 rounding).  0 <= n <
 * 2^31.  ENV_EINVAL on bad sizes, NULL arrays, op_in == op_out. */
int gr_opinion_step(int64_t n, int64_t n_edges, const int64_t *row_ptr, const int32_t *col,
                    const float *weight, float threshold, float strength, const float *op_in,
                    float *op_out, int lanes, void *stream);

/* -------------------------------------------------------------- serving */

/* Continuous-batching server.  The paper serves nothing: this is a systems
 * pattern round its loop of Sec. 4.3 and Fig. 5 (the shared policy acts on
 * every agent's view, the env steps, state stays in device memory as in
 * Sec. 2.2), with episodes of different sizes joining and leaving a running
 * batch.  `arena` (device, `arena_bytes`) is the HBM
 * budget: each admitted request's env workspace, view/action/reward rows and
 * the tick's batch scratch are carved from it.  At most max_slots requests
 * run at once.  All requests share `pol`: their view row length d must
 * equal pol's in, and every request has the sector count of the first one
 * submitted (ENV_EINVAL otherwise).  Fields of view may differ.
 */
int srv_create(void *arena, size_t arena_bytes, int max_slots, pol_t *pol,
               void *stream, srv_t **out);
void srv_destroy(srv_t *srv);

/* Queue an episode request: parameters (Sec. 4.1), initial state (host FP32
 * x, y, th, s, each [n], copied before return) and episode length.  Never blocks; *id receives the request
 * id.  Returns ENV_OK when admitted at once, ENV_EAGAIN when queued (no slot
 * or no memory yet), ENV_ENOMEM when the request could never fit. */
int srv_submit(srv_t *srv, const env_params_t *p, const float *x, const float *y,
               const float *th, const float *s, int steps, int64_t *id);

/* One serving tick, one step of Fig. 5's loop for every running episode:
 * admit queued requests that now fit (in arrival order; a
 * later request that fits may pass a waiting one, but once the head of the
 * queue has waited 32 ticks nothing passes it until it is admitted), run one closed-loop
 * batched step over all running requests, retire those that finished.
 * *n_running / *agents receive the number of requests and agents stepped.
 * Synchronises the stream at the end of the tick. */
int srv_tick(srv_t *srv, int32_t *n_running, int64_t *agents);

/* *state: 0 queued, 1 running, 2 finished; *steps_done: steps so far.
 * ENV_ENOTFOUND for an unknown id (or one whose result was taken). */
int srv_poll(srv_t *srv, int64_t id, int32_t *state, int32_t *steps_done);

/* Per-agent FP64 returns of a finished request (host [n]; the undiscounted
 * sum of Eq. (1)'s rewards over the episode, agent order); frees its record.
 * ENV_ESTATE while it is queued or runs, ENV_ENOTFOUND for an unknown id,
 * ENV_EINVAL for a wrong n. */
int srv_result(srv_t *srv, int64_t id, double *returns_host, int64_t n);

/* Arena bytes one request with these parameters occupies (0 if invalid). */
size_t srv_request_bytes(const env_params_t *p);

#if defined(__GNUC__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif

#endif /* FLOCKENV_H */
