// flock_api.cpp -- the C ABI declared in include/flockenv.h: parameter
// validation, cell-grid geometry, workspace carving and the env / batch
// objects.  Every device computation is a kernel in flock_kernels.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "flock_internal.h"

using namespace flock;

// ----------------------------------------------------------------- errors

namespace {
thread_local std::string g_err;

int vfail(int code, const char *fmt, va_list ap) {
    char buf[512];
    vsnprintf(buf, sizeof(buf), fmt, ap);
    g_err = buf;
    return code;
}

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(code, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(ENV_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite(float v) { return isfinite(v) != 0; }

// Largest agent count per env and per batch (row indices are int32).
constexpr int64_t kMaxAgents = int64_t(1) << 26;
constexpr int64_t kMaxBatchAgents = int64_t(1) << 30;
// Cell indices are int32 and the two-level scan's tile count must fit a grid.
constexpr int64_t kMaxBatchCells = int64_t(1) << 28;

int check_params(const env_params_t *p) {
    if (!p) return fail(ENV_EINVAL, "params is NULL");
    if (p->n_agents < 0 || p->n_agents > kMaxAgents)
        return fail(ENV_EINVAL, "n_agents %d outside [0, 2^26]", p->n_agents);
    if (!finite(p->box) || !(p->box > 0.0f)) return fail(ENV_EINVAL, "box must be finite and > 0");
    if (!finite(p->radius) || !(p->radius > 0.0f))
        return fail(ENV_EINVAL, "radius must be finite and > 0");
    if (!(p->radius < 0.5f * p->box))
        return fail(ENV_EINVAL, "radius %g must be < box/2 (%g)", p->radius, 0.5f * p->box);
    if (!finite(p->collide) || p->collide < 0.0f || p->collide > p->radius)
        return fail(ENV_EINVAL, "collide must be in [0, radius]");
    if (p->sectors < 1 || p->sectors > 256) return fail(ENV_EINVAL, "sectors must be in [1, 256]");
    if (!finite(p->r_nb) || !finite(p->r_col)) return fail(ENV_EINVAL, "rewards must be finite");
    if (!finite(p->max_turn) || p->max_turn < 0.0f || !finite(p->max_dspeed) || p->max_dspeed < 0.0f)
        return fail(ENV_EINVAL, "max_turn and max_dspeed must be finite and >= 0");
    if (!finite(p->s_min) || !finite(p->s_max) || p->s_min < 0.0f || p->s_min > p->s_max)
        return fail(ENV_EINVAL, "need 0 <= s_min <= s_max");
    if (p->cell_reach < 0 || p->cell_reach > 2) return fail(ENV_EINVAL, "cell_reach must be 0, 1 or 2");
    if (p->flags & ~(ENV_FLAG_COUNTS | ENV_FLAG_SPEED_OBS | ENV_FLAG_TAG))
        return fail(ENV_EINVAL, "unknown flags 0x%x", p->flags);
    if (p->flags & ENV_FLAG_TAG) {
        if (p->n_chasers < 0 || p->n_chasers > p->n_agents)
            return fail(ENV_EINVAL, "n_chasers must be in [0, n_agents]");
        if (!finite(p->r_catch)) return fail(ENV_EINVAL, "r_catch must be finite");
        if (p->sectors > 128) return fail(ENV_EINVAL, "tag envs take at most 128 sectors per channel");
    }
    if (!finite(p->fov) || p->fov < 0.0f || p->fov > kTwoPiF)
        return fail(ENV_EINVAL, "fov must be 0 (full view) or in (0, 2 pi]");
    return ENV_OK;
}


bool valid_lanes(int lanes) { return lanes == 1 || lanes == 4 || lanes == 16 || lanes == 64; }

struct Geometry {
    int ncx, ncy, reach;
    float cw, ch, inv_cx, inv_cy, marg;
};

// Rows per column: a column's candidates are the rows within the vision
// range of the agent's y, so rows far narrower than the range trim the
// stencil to the disc more closely; a run costs the same however many rows
// it spans.
constexpr int kRowsPerColumnWidth = 4;

// Columns are at least radius/reach wide after FP32 rounding of the cell
// boundaries: floor(x * inv_cx) moves a boundary by at most box * 2^-23,
// so the nominal width carries a margin of 4 * box * 2^-23.  The grid is
// also capped near sqrt(4n) columns so empty boxes stay cheap (wider
// columns only add candidates).  Fewer than 2 reach + 1 columns would visit
// a column twice, so such boxes fall back to one cell and all pairs.  Each
// column holds kRowsPerColumnWidth times as many rows; the sweep widens its
// row bounds by marg = box * 2^-20, well above the rounding of the row
// assignment, of the bounds themselves and of the pair test.
Geometry geometry(const env_params_t &p) {
    Geometry g{1, 1, 0, p.box, p.box, 0.0f, 0.0f, 0.0f};
    const double L = p.box, R = p.radius;
    const double margin = 4.0 * L * ldexp(1.0, -23);
    const int64_t cap = (int64_t)ceil(sqrt(4.0 * (double)(p.n_agents > 0 ? p.n_agents : 1))) + 3;
    for (int r = (p.cell_reach == 0 ? 1 : p.cell_reach); r >= 1; --r) {
        int64_t nc = (int64_t)floor(L / (R / r + margin));
        if (nc > cap) nc = cap;
        if (nc > 8192) nc = 8192;
        if (nc >= 2 * r + 1) {
            g.ncx = (int)nc;
            g.ncy = (int)nc * kRowsPerColumnWidth;
            g.reach = r;
            g.cw = (float)(L / (double)g.ncx);
            g.ch = (float)(L / (double)g.ncy);
            g.inv_cx = (float)((double)g.ncx / L);
            g.inv_cy = (float)((double)g.ncy / L);
            g.marg = (float)(L * ldexp(1.0, -20));
            return g;
        }
    }
    return g;
}

DevEnv make_desc(const env_params_t &p, const Geometry &gm) {
    DevEnv d;
    memset(&d, 0, sizeof(d));
    d.n = p.n_agents;
    d.ncx = gm.ncx;
    d.ncy = gm.ncy;
    d.reach = gm.reach;
    d.box = p.box;
    d.inv_cx = gm.inv_cx;
    d.inv_cy = gm.inv_cy;
    d.cw = gm.cw;
    d.marg = gm.marg;
    d.r2 = p.radius * p.radius;
    d.c2 = p.collide * p.collide;
    d.inv_radius = (float)(1.0 / (double)p.radius);
    d.r_nb = p.r_nb;
    d.r_col = p.r_col;
    d.max_turn = p.max_turn;
    d.max_dspeed = p.max_dspeed;
    d.s_min = p.s_min;
    d.s_max = p.s_max;
    d.tag = (p.flags & ENV_FLAG_TAG) ? 1 : 0;
    d.n_chasers = d.tag ? p.n_chasers : 0;
    d.r_catch = p.r_catch;
    if (full_view(p)) {
        d.fov_half = 0.0f;
        d.fov_t = 1.0f;
        d.sec_scale = (float)p.sectors;
    } else {
        const double t = (double)p.fov / (2.0 * M_PI);  // arc in turns
        d.fov_t = (float)t;
        d.fov_half = 0.5f * d.fov_t;
        d.sec_scale = (float)((double)p.sectors / (double)d.fov_t);
    }
    return d;
}

// Device arrays of one env: two cell-order record buffers (ping-pong), the
// agent-order counts and the scratch of its own (batch-of-one) step.
struct EnvLayout {
    float4 *rec[2];
    int32_t *id[2];
    double *ret[2];
    int32_t *nb, *col;
    SortArrays sort;
    size_t bytes;
};

// Strips of an env's own step (a plan of one env), 0 when the strip sort is
// not allowed for it.
int64_t env_own_strips(const env_params_t &p, const Geometry &gm) {
    DevEnv d = make_desc(p, gm);
    if (!strips_allowed(d)) return 0;
    DevEnv *tabs[1] = {&d};
    return assign_strips(tabs, 1, 1, p.n_agents, nullptr);
}

EnvLayout carve_env(char *base, const env_params_t &p, const Geometry &gm) {
    EnvLayout l;
    Carver cv{base, 0};
    const int64_t n = p.n_agents;
    for (int b = 0; b < 2; ++b) {
        l.rec[b] = cv.take<float4>(n);
        l.id[b] = cv.take<int32_t>(n);
        l.ret[b] = cv.take<double>(n);
    }
    const bool counts = (p.flags & ENV_FLAG_COUNTS) != 0;
    l.nb = counts ? cv.take<int32_t>(n) : nullptr;
    l.col = counts ? cv.take<int32_t>(n) : nullptr;
    carve_sort(cv, n, (int64_t)gm.ncx * gm.ncy, 1, &l.sort, env_own_strips(p, gm));
    l.bytes = align_up(cv.off, 256);
    return l;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

bool flock::full_view(const env_params_t &p) { return p.fov == 0.0f || p.fov >= kTwoPiF; }
int flock::obs_dim_of(const env_params_t &p) {
    const int channels = (p.flags & ENV_FLAG_TAG) ? 2 : 1;
    return channels * p.sectors + ((p.flags & ENV_FLAG_SPEED_OBS) ? 1 : 0);
}

int flock::set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(code, fmt, ap);
    va_end(ap);
    return code;
}

// ------------------------------------------------------------------ objects

struct flock_env {
    env_params_t p;
    Geometry gm;
    EnvLayout lay;
    StepPlan plan;          // its own step: a batch of one
    DevEnv scalars;         // descriptor without buffer pointers
    DevEnv own[2];          // own tables: [b] has buffer b current
    int32_t base_host[2];   // {0, n}
    int parity = 0;         // index of the current record buffer
    uint64_t gen = 0;       // bumped by every call that changes the state
    bool sorted = false;    // records in cell order (after a sort; not after set_state)
    bool has_state = false;
    bool reset_done = false;
    bool uploaded = false;
};

namespace {

DevEnv orient(const env_t *e, int cur) {
    DevEnv d = e->scalars;
    d.rec_cur = e->lay.rec[cur];
    d.rec_nxt = e->lay.rec[cur ^ 1];
    d.id_cur = e->lay.id[cur];
    d.id_nxt = e->lay.id[cur ^ 1];
    d.ret_cur = e->lay.ret[cur];
    d.ret_nxt = e->lay.ret[cur ^ 1];
    return d;
}

int upload_own(env_t *e, hipStream_t s) {
    if (e->uploaded) return ENV_OK;
    hipError_t err = hipMemcpyAsync(e->lay.sort.envs[0], &e->own[0], sizeof(DevEnv),
                                    hipMemcpyHostToDevice, s);
    if (err == hipSuccess)
        err = hipMemcpyAsync(e->lay.sort.envs[1], &e->own[1], sizeof(DevEnv),
                             hipMemcpyHostToDevice, s);
    if (err == hipSuccess)
        err = hipMemcpyAsync(e->lay.sort.base, e->base_host, sizeof(e->base_host),
                             hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = launch_clear(e->plan, s);
    if (err != hipSuccess) return hip_fail(err, "env descriptor upload");
    e->uploaded = true;
    return ENV_OK;
}

}  // namespace

// An instantiated graph and the launch arguments it was captured with.
struct GraphCache {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<uint64_t> key;
};

struct flock_batch {
    std::vector<env_t *> envs;
    std::vector<int> base_par;       // env parities the tables were built for
    std::vector<DevEnv> tab[2];      // [t]: env k has buffer base_par[k] ^ t current
    std::vector<int32_t> base;
    std::vector<int64_t> off;
    std::vector<int32_t> strip_env;  // env of each strip (strip sort)
    StepPlan plan;
    bool uploaded = false;
    GraphCache gc[2];                // K-step graphs by starting table
    GraphCache rgc[2];               // rollout graphs by starting table
    hipEvent_t events[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    // env_step_policy's next actions, computed inside its view sweep: valid
    // for the next call with the same policy and obs while no env changed.
    bool fuse_policy = false;        // env_batch_set_policy_fusion
    float2 *act_next = nullptr;      // [G] in the workspace
    bool next_valid = false;
    const void *next_pol = nullptr;
    const float *next_obs = nullptr;
    std::vector<uint64_t> next_gen;
};

namespace flock {

int validate_params(const env_params_t *p) { return check_params(p); }

DevEnv env_descriptor(const env_t *env, int flip) { return orient(env, env->parity ^ (flip & 1)); }

int64_t env_cell_count(const env_t *env) { return (int64_t)env->gm.ncx * env->gm.ncy; }

int64_t cell_count_for(const env_params_t &p) {
    const Geometry g = geometry(p);
    return (int64_t)g.ncx * g.ncy;
}

int64_t column_count_for(const env_params_t &p) { return geometry(p).ncx; }

// The stencil's area before trimming to the disc: 2 reach + 1 columns, each
// 2 radius + one row high.
double env_candidates_per_agent(const env_t *env) {
    const double n = env->p.n_agents;
    const Geometry &g = env->gm;
    if (g.ncx == 1) return n;
    const double L = env->p.box;
    const double area = (2.0 * g.reach + 1.0) * g.cw * (2.0 * env->p.radius + g.ch);
    return n * std::min(1.0, area / (L * L));
}

// One lane per agent suits a few dozen candidates.  Beyond that a lane group
// per agent keeps the lanes busy; with many sectors (v > 32) one lane per
// agent also needs v words of LDS per lane, which caps occupancy, so groups
// of 16 win early.  Measured on MI355X: 30 candidates, v = 16 -> 1;
// ~500, v = 16 -> 4; 111 and 1,111, v = 128 -> 16.
int auto_lanes(double cand, int v, int64_t agents) {
    // sparse neighbourhoods: one lane per agent, unless there are so few
    // agents that wider groups keep more CUs busy (one-env steps with about
    // 20 candidates per agent: 5,000 agents 27 us at one lane, 23 us at 64;
    // 1,000 agents 23 and 18 us; 16,000 agents 32 us at one lane, 29 at 16;
    // from 32,000 agents one lane is fastest)
    if (cand < 64.0) {
        if (agents * 64 <= (int64_t(1) << 19)) return 64;
        if (agents * 16 <= (int64_t(1) << 18)) return 16;
        return 1;
    }
    int lanes = v > 32 ? 16 : (cand < 1024.0 ? 4 : 16);
    // few agents with dense neighbourhoods: wider groups keep the GPU busy
    // (one 16,000-agent env of about 1,000 candidates each steps 20 % faster
    // with 64 lanes than with 16)
    if (cand >= 256.0 && agents * lanes < (int64_t(1) << 19)) lanes = 64;
    return lanes;
}

const env_params_t &env_params(const env_t *env) { return env->p; }

int env_parity(const env_t *env) { return env->parity; }

void env_advance(env_t *env, int steps) {
    env->parity ^= (steps & 1);
    env->sorted = true;
    ++env->gen;
}

bool env_sorted(const env_t *env) { return env->sorted; }

int env_load_host_state(env_t *env, const float *x, const float *y, const float *th,
                        const float *s_, hipStream_t s) {
    const int n = env->p.n_agents;
    env->has_state = true;
    env->sorted = false;
    ++env->gen;
    if (n == 0) return ENV_OK;
    // Stage the agent-order arrays in the next buffer's record area (free
    // until the next step) and load them into the current buffer.
    float *stage = reinterpret_cast<float *>(env->lay.rec[env->parity ^ 1]);
    const size_t b = (size_t)n * sizeof(float);
    hipError_t e = hipMemcpyAsync(stage, x, b, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(stage + n, y, b, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(stage + 2 * (size_t)n, th, b, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(stage + 3 * (size_t)n, s_, b, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_load_state(stage, stage + n, stage + 2 * (size_t)n, stage + 3 * (size_t)n,
                              env->lay.rec[env->parity], env->lay.id[env->parity], n, s);
    if (e != hipSuccess) return hip_fail(e, "state upload");
    return ENV_OK;
}

int env_returns_to(env_t *env, double *out, hipStream_t s) {
    hipError_t e = launch_store_returns(env->lay.ret[env->parity], env->lay.id[env->parity], out,
                                        env->p.n_agents, s);
    if (e != hipSuccess) return hip_fail(e, "returns");
    return ENV_OK;
}

size_t sort_scratch_bytes(int64_t G, int64_t C, int E, int64_t S) {
    Carver cv{nullptr, 0};
    SortArrays a;
    carve_sort(cv, G, C, E, &a, S);
    return align_up(cv.off, 256);
}

}  // namespace flock

static void drop_graph(GraphCache &gc) {
    if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
    if (gc.graph) (void)hipGraphDestroy(gc.graph);
    gc = GraphCache{};
}

static void drop_graphs(env_batch_t *b) {
    for (auto &gc : b->gc) drop_graph(gc);
    for (auto &gc : b->rgc) drop_graph(gc);
}

// Capture what `enqueue` launches on `s` into `gc`, unless gc already holds a
// graph captured with the same key.
template <typename F>
static int capture_graph(GraphCache &gc, std::vector<uint64_t> key, hipStream_t s, F enqueue) {
    if (gc.exec && gc.key == key) return ENV_OK;
    drop_graph(gc);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    const hipError_t le = enqueue();
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le != hipSuccess ? le : e, "graph capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    gc.exec = exec;
    gc.graph = graph;
    gc.key = std::move(key);
    return ENV_OK;
}

static uint64_t key_of(const void *p) { return (uint64_t)reinterpret_cast<uintptr_t>(p); }

extern "C" {

const char *env_last_error(void) { return g_err.c_str(); }

size_t env_workspace_bytes(const env_params_t *p) {
    if (check_params(p) != ENV_OK) return 0;
    const Geometry gm = geometry(*p);
    return carve_env(nullptr, *p, gm).bytes;
}

int env_create(const env_params_t *p, void *workspace, size_t bytes, env_t **out) {
    int rc = check_params(p);
    if (rc != ENV_OK) return rc;
    if (!out) return fail(ENV_EINVAL, "out is NULL");
    if (!workspace) return fail(ENV_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(ENV_EINVAL, "workspace must be 256-byte aligned");
    const Geometry gm = geometry(*p);
    const size_t need = carve_env(nullptr, *p, gm).bytes;
    if (bytes < need) return fail(ENV_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, need);
    env_t *e = new env_t;
    e->p = *p;
    e->gm = gm;
    e->lay = carve_env(static_cast<char *>(workspace), *p, gm);
    e->scalars = make_desc(*p, gm);
    e->scalars.nb = e->lay.nb;
    e->scalars.col = e->lay.col;
    const int64_t own_strips = env_own_strips(*p, gm);
    if (own_strips > 0) {
        DevEnv *tabs[1] = {&e->scalars};
        assign_strips(tabs, 1, 1, p->n_agents, nullptr);
    }
    e->own[0] = orient(e, 0);
    e->own[1] = orient(e, 1);
    e->base_host[0] = 0;
    e->base_host[1] = p->n_agents;
    e->plan.a = e->lay.sort;
    e->plan.n_envs = 1;
    e->plan.G = p->n_agents;
    e->plan.C = (int64_t)gm.ncx * gm.ncy;
    e->plan.v = p->sectors;
    e->plan.obs_dim = obs_dim_of(*p);
    e->plan.fov = full_view(*p) ? 0 : 1;
    e->plan.tag = (p->flags & ENV_FLAG_TAG) ? 1 : 0;
    e->plan.lanes = auto_lanes(env_candidates_per_agent(e), p->sectors, p->n_agents);
    e->plan.max_env_cells = e->plan.C;
    e->plan.env_sort_recs = 0;  // one env: the multi-block kernels fill the GPU better
    e->plan.strips = (int)own_strips;
    if (own_strips > 0) plan_strip_launch(&e->plan, &e->scalars, 1);
    e->plan.scan_blocks = scan_blocks_for(e->plan.C, e->plan.C);
    *out = e;
    g_err.clear();
    return ENV_OK;
}

void env_destroy(env_t *env) { delete env; }

int env_geometry(const env_t *env, int32_t *ncx, int32_t *ncy, int32_t *reach, float *cell_w,
                 float *cell_h) {
    if (!env) return fail(ENV_EINVAL, "env is NULL");
    if (ncx) *ncx = env->gm.ncx;
    if (ncy) *ncy = env->gm.ncy;
    if (reach) *reach = env->gm.reach;
    if (cell_w) *cell_w = env->gm.cw;
    if (cell_h) *cell_h = env->gm.ch;
    return ENV_OK;
}

int env_set_sweep_lanes(env_t *env, int lanes) {
    if (!env) return fail(ENV_EINVAL, "env is NULL");
    if (lanes != 0 && !valid_lanes(lanes)) return fail(ENV_EINVAL, "lanes must be 0, 1, 4, 16 or 64");
    env->plan.lanes =
        lanes ? lanes : auto_lanes(env_candidates_per_agent(env), env->p.sectors, env->p.n_agents);
    return ENV_OK;
}

int env_set_state(env_t *env, const float *x, const float *y, const float *th, const float *s,
                  void *stream) {
    if (!env) return fail(ENV_EINVAL, "env is NULL");
    const int n = env->p.n_agents;
    if (n > 0 && (!x || !y || !th || !s)) return fail(ENV_EINVAL, "state pointer is NULL");
    hipError_t e = launch_load_state(x, y, th, s, env->lay.rec[env->parity],
                                     env->lay.id[env->parity], n, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "env_set_state");
    env->has_state = true;
    env->sorted = false;
    ++env->gen;
    return ENV_OK;
}

int env_get_state(env_t *env, float *x, float *y, float *th, float *s, void *stream) {
    if (!env) return fail(ENV_EINVAL, "env is NULL");
    const int n = env->p.n_agents;
    if (n > 0 && (!x || !y || !th || !s)) return fail(ENV_EINVAL, "state pointer is NULL");
    if (!env->has_state) return fail(ENV_ESTATE, "env has no state yet");
    hipError_t e = launch_store_state(env->lay.rec[env->parity], env->lay.id[env->parity], x, y,
                                      th, s, n, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "env_get_state");
    return ENV_OK;
}

int env_reset(env_t *env, float *obs, void *stream) {
    if (!env) return fail(ENV_EINVAL, "env is NULL");
    if (!env->has_state) return fail(ENV_ESTATE, "env_reset before env_set_state");
    const int n = env->p.n_agents;
    if (n > 0 && !obs) return fail(ENV_EINVAL, "obs is NULL");
    hipStream_t s = as_stream(stream);
    int rc = upload_own(env, s);
    if (rc != ENV_OK) return rc;
    hipError_t e = launch_zero_f64(env->lay.ret[env->parity], n, s);
    if (e != hipSuccess) return hip_fail(e, "env_reset: zero returns");
    // The sense-only pass yields no reward: the episode's first reward comes
    // with the first step.  It sorts the records into cell order.
    env->plan.strip_now = env->sorted ? 1 : 0;
    e = launch_step(env->plan, env->parity, 0, nullptr, obs, nullptr, 0, s);
    if (e != hipSuccess) return hip_fail(e, "env_reset: sense");
    if (n > 0) env->parity ^= 1;
    env->reset_done = true;
    env->sorted = true;
    ++env->gen;
    return ENV_OK;
}

int env_step(env_t *env, const float *act, float *obs, float *reward, void *stream) {
    if (!env) return fail(ENV_EINVAL, "env is NULL");
    if (!env->reset_done) return fail(ENV_ESTATE, "env_step before env_reset");
    const int n = env->p.n_agents;
    if (n > 0 && (!act || !obs || !reward)) return fail(ENV_EINVAL, "act/obs/reward is NULL");
    env->plan.strip_now = env->sorted ? 1 : 0;
    hipError_t e = launch_step(env->plan, env->parity, 1, act, obs, reward, 1, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "env_step");
    if (n > 0) env->parity ^= 1;
    env->sorted = true;
    ++env->gen;
    return ENV_OK;
}

int env_get_counts(env_t *env, int32_t *n_nb, int32_t *n_col, void *stream) {
    if (!env) return fail(ENV_EINVAL, "env is NULL");
    if (!(env->p.flags & ENV_FLAG_COUNTS)) return fail(ENV_ESTATE, "env created without ENV_FLAG_COUNTS");
    if (!env->reset_done) return fail(ENV_ESTATE, "no step has run yet");
    const int n = env->p.n_agents;
    if (n > 0 && (!n_nb || !n_col)) return fail(ENV_EINVAL, "count pointer is NULL");
    hipError_t e = launch_copy_i32(env->lay.nb, n_nb, n, as_stream(stream));
    if (e == hipSuccess) e = launch_copy_i32(env->lay.col, n_col, n, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "env_get_counts");
    return ENV_OK;
}

int env_get_returns(env_t *env, double *ret, void *stream) {
    if (!env) return fail(ENV_EINVAL, "env is NULL");
    if (!env->reset_done) return fail(ENV_ESTATE, "env_get_returns before env_reset");
    const int n = env->p.n_agents;
    if (n > 0 && !ret) return fail(ENV_EINVAL, "ret is NULL");
    return env_returns_to(env, ret, as_stream(stream));
}

int env_set_returns(env_t *env, const double *ret, void *stream) {
    if (!env) return fail(ENV_EINVAL, "env is NULL");
    if (!env->reset_done) return fail(ENV_ESTATE, "env_set_returns before env_reset");
    const int n = env->p.n_agents;
    if (n > 0 && !ret) return fail(ENV_EINVAL, "ret is NULL");
    hipError_t e = launch_load_returns(ret, env->lay.id[env->parity], env->lay.ret[env->parity], n,
                                       as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "env_set_returns");
    return ENV_OK;
}

}  // extern "C"

// ------------------------------------------------------- static step scratch
//
// env_step_static takes the sort scratch of its step (cell keys, ranks, moved
// records, candidate positions, cell counts and starts, descriptor tables)
// from `scratch`, one array per GPU that the library runs on, held until the
// process ends, instead of from the env's workspace.  In host code the
// array's name stands for a host-side shadow, not a device address: kernels
// only ever get the per-device address hipGetSymbolAddress returns.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];

// Device address of `scratch` on the current device (looked up once per device).
int static_scratch(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(ENV_EINVAL, "device %d: the static scratch is tracked for devices 0..%d", dev,
                    kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(ENV_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return ENV_OK;
}
}  // namespace

extern "C" {

size_t env_static_scratch_bytes(void) { return kStaticScratchBytes; }

int env_step_static(env_t *env, const float *act, float *obs, float *reward, void *stream) {
    if (!env) return fail(ENV_EINVAL, "env is NULL");
    const size_t need = sort_scratch_bytes(env->plan.G, env->plan.C, 1, env->plan.strips);
    if (need > kStaticScratchBytes)
        return fail(ENV_ENOMEM,
                    "env_step_static: a step of %lld agents over %lld cells needs %zu bytes of "
                    "scratch; the static array holds %zu (use env_step)",
                    (long long)env->plan.G, (long long)env->plan.C, need, kStaticScratchBytes);
    if (!env->reset_done) return fail(ENV_ESTATE, "env_step_static before env_reset");
    const int n = env->p.n_agents;
    if (n > 0 && (!act || !obs || !reward)) return fail(ENV_EINVAL, "act/obs/reward is NULL");
    if (n == 0) return ENV_OK;
    void *base = nullptr;
    int rc = static_scratch(&base);
    if (rc != ENV_OK) return rc;
    StepPlan p = env->plan;
    Carver cv{static_cast<char *>(base), 0};
    carve_sort(cv, p.G, p.C, 1, &p.a, p.strips);
    p.strip_now = env->sorted ? 1 : 0;
    hipStream_t s = as_stream(stream);
    hipError_t e = launch_bind_one(p, env->own[0], env->own[1], n, s);
    if (e == hipSuccess) e = launch_step(p, env->parity, 1, act, obs, reward, 1, s);
    if (e != hipSuccess) return hip_fail(e, "env_step_static");
    env->parity ^= 1;
    env->sorted = true;
    ++env->gen;
    return ENV_OK;
}

// ------------------------------------------------------------------- batch

static int batch_layout(env_t *const *envs, int n_envs, std::vector<int32_t> *base,
                        std::vector<int64_t> *off, int64_t *G, int64_t *C, int *v,
                        int *obs_dim = nullptr, int *fov = nullptr) {
    if (!envs || n_envs < 1) return fail(ENV_EINVAL, "need at least one env");
    int64_t g = 0, c = 0;
    for (int k = 0; k < n_envs; ++k) {
        const env_t *e = envs[k];
        if (!e) return fail(ENV_EINVAL, "env %d is NULL", k);
        if (e->p.sectors != envs[0]->p.sectors)
            return fail(ENV_EINVAL, "env %d has %d sectors, env 0 has %d", k, e->p.sectors,
                        envs[0]->p.sectors);
        if ((e->p.flags & ENV_FLAG_TAG) != (envs[0]->p.flags & ENV_FLAG_TAG))
            return fail(ENV_EINVAL, "env %d and env 0 differ in ENV_FLAG_TAG", k);
        if (obs_dim_of(e->p) != obs_dim_of(envs[0]->p))
            return fail(ENV_EINVAL, "env %d and env 0 differ in ENV_FLAG_SPEED_OBS", k);
        if (fov && !full_view(e->p)) *fov = 1;
        if (base) base->push_back((int32_t)g);
        if (off) off->push_back(g);
        g += e->p.n_agents;
        c += (int64_t)e->gm.ncx * e->gm.ncy;
        if (g > kMaxBatchAgents || c > kMaxBatchCells)
            return fail(ENV_EINVAL, "batch exceeds 2^30 agents or 2^28 cells");
    }
    if (base) base->push_back((int32_t)g);
    if (off) off->push_back(g);
    *G = g;
    *C = c;
    *v = envs[0]->p.sectors;
    if (obs_dim) *obs_dim = obs_dim_of(envs[0]->p);
    return ENV_OK;
}

// Strips of a batch's envs (the strip sort), 0 when some env does not allow it.
static int64_t batch_strips(env_t *const *envs, int n_envs, int64_t G,
                            std::vector<int32_t> *strip_env) {
    std::vector<DevEnv> d(n_envs);
    for (int k = 0; k < n_envs; ++k) {
        d[k] = envs[k]->scalars;
        if (!strips_allowed(d[k])) return 0;
    }
    DevEnv *tabs[1] = {d.data()};
    return assign_strips(tabs, 1, n_envs, G, strip_env);
}

size_t env_batch_workspace_bytes(env_t *const *envs, int n_envs) {
    int64_t G, C;
    int v;
    if (batch_layout(envs, n_envs, nullptr, nullptr, &G, &C, &v) != ENV_OK) return 0;
    const int64_t S = batch_strips(envs, n_envs, G, nullptr);
    return sort_scratch_bytes(G, C, n_envs, S) + align_up((size_t)G * sizeof(float2), 256);
}

static int batch_auto_lanes(const std::vector<env_t *> &envs) {
    double cand = 0.0, n = 0.0;
    for (const env_t *e : envs) {
        cand += env_candidates_per_agent(e) * e->p.n_agents;
        n += e->p.n_agents;
    }
    return auto_lanes(n > 0.0 ? cand / n : 0.0, envs.empty() ? 1 : envs[0]->p.sectors,
                      (int64_t)n);
}

int env_batch_create(env_t *const *envs, int n_envs, void *ws, size_t bytes, env_batch_t **out) {
    if (!out) return fail(ENV_EINVAL, "out is NULL");
    if (!ws) return fail(ENV_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(ENV_EINVAL, "workspace must be 256-byte aligned");
    env_batch_t *b = new env_batch_t;
    int64_t G, C;
    int v, obs_dim = 0, fov = 0;
    int rc = batch_layout(envs, n_envs, &b->base, &b->off, &G, &C, &v, &obs_dim, &fov);
    if (rc != ENV_OK) {
        delete b;
        return rc;
    }
    for (int k = 0; k < n_envs; ++k) {
        if (!envs[k]->reset_done) {
            delete b;
            return fail(ENV_ESTATE, "env %d has not been reset", k);
        }
    }
    Carver cv{static_cast<char *>(ws), 0};
    const int64_t S = batch_strips(envs, n_envs, G, &b->strip_env);
    carve_sort(cv, G, C, n_envs, &b->plan.a, S);
    b->act_next = cv.take<float2>((size_t)G);
    if (bytes < align_up(cv.off, 256)) {
        delete b;
        return fail(ENV_ENOMEM, "batch workspace has %zu bytes, needs %zu", bytes,
                    align_up(cv.off, 256));
    }
    b->envs.assign(envs, envs + n_envs);
    b->base_par.assign(n_envs, -1);
    b->plan.n_envs = n_envs;
    b->plan.G = G;
    b->plan.C = C;
    b->plan.v = v;
    b->plan.obs_dim = obs_dim;
    b->plan.fov = fov;
    b->plan.tag = (envs[0]->p.flags & ENV_FLAG_TAG) ? 1 : 0;
    b->plan.lanes = batch_auto_lanes(b->envs);
    int64_t max_cells = 0, max_agents = 0;
    for (const env_t *e : b->envs) {
        max_cells = std::max(max_cells, env_cell_count(e));
        max_agents = std::max(max_agents, (int64_t)e->p.n_agents);
    }
    b->plan.max_env_cells = max_cells;
    b->plan.env_sort_recs = env_sort_recs_for(n_envs, max_agents, max_cells);
    b->plan.scan_blocks = scan_blocks_for(C, max_cells);
    b->plan.strips = (int)S;
    if (S > 0) {
        std::vector<DevEnv> d(n_envs);
        for (int k = 0; k < n_envs; ++k) d[k] = envs[k]->scalars;
        DevEnv *tabs[1] = {d.data()};
        assign_strips(tabs, 1, n_envs, G, nullptr);
        plan_strip_launch(&b->plan, d.data(), n_envs);
    }
    *out = b;
    return ENV_OK;
}



void env_batch_destroy(env_batch_t *b) {
    if (!b) return;
    drop_graphs(b);
    for (auto &ev : b->events)
        if (ev) (void)hipEventDestroy(ev);
    delete b;
}

int env_batch_set_sweep_lanes(env_batch_t *b, int lanes) {
    if (!b) return fail(ENV_EINVAL, "batch is NULL");
    if (lanes != 0 && !valid_lanes(lanes)) return fail(ENV_EINVAL, "lanes must be 0, 1, 4, 16 or 64");
    const int want = lanes ? lanes : batch_auto_lanes(b->envs);
    if (want != b->plan.lanes) {
        drop_graphs(b);
        b->plan.lanes = want;
    }
    return ENV_OK;
}

int env_batch_set_policy_fusion(env_batch_t *b, int on) {
    if (!b) return fail(ENV_EINVAL, "batch is NULL");
    const bool want = on != 0;
    if (want != b->fuse_policy) {
        drop_graphs(b);
        b->fuse_policy = want;
        b->next_valid = false;
    }
    return ENV_OK;
}

int env_batch_set_strip_wait(env_batch_t *b, int polls) {
    if (!b) return fail(ENV_EINVAL, "batch is NULL");
    if (polls < 0) return fail(ENV_EINVAL, "polls must be >= 0");
    if (polls != b->plan.strip_wait) {
        drop_graphs(b);
        b->plan.strip_wait = polls;
    }
    return ENV_OK;
}

int env_batch_get_sweep_lanes(const env_batch_t *b, int32_t *lanes) {
    if (!b || !lanes) return fail(ENV_EINVAL, "NULL argument");
    *lanes = b->plan.lanes;
    return ENV_OK;
}

int env_batch_offsets(const env_batch_t *b, int64_t *off) {
    if (!b || !off) return fail(ENV_EINVAL, "NULL argument");
    for (size_t k = 0; k < b->off.size(); ++k) off[k] = b->off[k];
    return ENV_OK;
}

// Make the device tables match the envs' current buffers; *table receives the
// table index of the next step.
static int batch_prepare(env_batch_t *b, hipStream_t s, int *table) {
    const int E = (int)b->envs.size();
    bool consistent = b->uploaded;
    const int t = b->envs[0]->parity ^ b->base_par[0];
    for (int k = 0; k < E && consistent; ++k)
        consistent = (b->envs[k]->parity ^ b->base_par[k]) == t;
    if (consistent) {
        *table = t & 1;
        return ENV_OK;
    }
    for (int f = 0; f < 2; ++f) {
        b->tab[f].clear();
        for (int k = 0; k < E; ++k) {
            DevEnv d = orient(b->envs[k], b->envs[k]->parity ^ f);
            d.agent_base = b->base[k];
            d.cell_base = 0;
            b->tab[f].push_back(d);
        }
    }
    int64_t c = 0;
    for (int k = 0; k < E; ++k) {
        b->tab[0][k].cell_base = b->tab[1][k].cell_base = (int32_t)c;
        c += (int64_t)b->envs[k]->gm.ncx * b->envs[k]->gm.ncy;
        b->base_par[k] = b->envs[k]->parity;
    }
    if (b->plan.strips > 0) {
        DevEnv *tabs[2] = {b->tab[0].data(), b->tab[1].data()};
        assign_strips(tabs, 2, E, b->plan.G, nullptr);
    }
    hipError_t e = hipSuccess;
    for (int f = 0; f < 2 && e == hipSuccess; ++f)
        e = hipMemcpyAsync(b->plan.a.envs[f], b->tab[f].data(), E * sizeof(DevEnv),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->plan.a.base, b->base.data(), b->base.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !b->uploaded && b->plan.strips > 0)
        e = hipMemcpyAsync(b->plan.a.strip_env, b->strip_env.data(),
                           b->strip_env.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !b->uploaded) e = launch_clear(b->plan, s);
    if (e != hipSuccess) return hip_fail(e, "batch upload");
    b->uploaded = true;
    drop_graphs(b);
    *table = 0;
    return ENV_OK;
}

// Every env of the batch swapped buffers `steps` times (empty envs too, so
// the parities of a batch stay in step).
static void batch_advance(env_batch_t *b, int steps) {
    for (env_t *e : b->envs) {
        e->parity ^= (steps & 1);
        e->sorted = true;
        ++e->gen;
    }
    b->next_valid = false;
}

// Whether this launch's first step may use the strip sort (every env's
// records in cell order); later steps of a launch always may.
static int batch_sorted(const env_batch_t *b) {
    for (const env_t *e : b->envs)
        if (!e->sorted) return 0;
    return 1;
}

int env_step_batched(env_batch_t *b, const float *act, float *obs, float *reward, void *stream) {
    if (!b) return fail(ENV_EINVAL, "batch is NULL");
    if (b->plan.G > 0 && (!act || !obs || !reward)) return fail(ENV_EINVAL, "act/obs/reward is NULL");
    hipStream_t s = as_stream(stream);
    int t;
    int rc = batch_prepare(b, s, &t);
    if (rc != ENV_OK) return rc;
    b->plan.strip_now = batch_sorted(b);
    hipError_t e = launch_step(b->plan, t, 1, act, obs, reward, 1, s);
    if (e != hipSuccess) return hip_fail(e, "env_step_batched");
    batch_advance(b, 1);
    return ENV_OK;
}

int env_step_batched_timed(env_batch_t *b, const float *act, float *obs, float *reward,
                           void *stream, float *phase_ms) {
    if (!b || !phase_ms) return fail(ENV_EINVAL, "NULL argument");
    if (b->plan.G > 0 && (!act || !obs || !reward)) return fail(ENV_EINVAL, "act/obs/reward is NULL");
    hipStream_t s = as_stream(stream);
    int t;
    int rc = batch_prepare(b, s, &t);
    if (rc != ENV_OK) return rc;
    if (!b->events[0]) {
        for (auto &ev : b->events) {
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        }
    }
    for (int k = 0; k < 4; ++k) phase_ms[k] = 0.0f;
    if (b->plan.G == 0) return ENV_OK;
    b->plan.strip_now = batch_sorted(b);
    hipError_t e = launch_step(b->plan, t, 1, act, obs, reward, 1, s, b->events);
    if (e != hipSuccess) return hip_fail(e, "env_step_batched_timed");
    batch_advance(b, 1);
    e = hipEventSynchronize(b->events[4]);
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
        e = hipEventElapsedTime(&phase_ms[k], b->events[k], b->events[k + 1]);
    if (e != hipSuccess) return hip_fail(e, "env_step_batched_timed");
    // the one-kernel sorts (per env, per strip) launch nothing for the scan and
    // scatter phases: what their events bracket is event overhead only
    if (b->plan.env_sort_recs > 0 || (b->plan.strips > 0 && b->plan.strip_now))
        phase_ms[1] = phase_ms[2] = 0.0f;
    return ENV_OK;
}

static int batch_capture(env_batch_t *b, int k_steps, const float *act, float *obs,
                         float *reward, void *stream, int *table) {
    if (!b) return fail(ENV_EINVAL, "batch is NULL");
    if (k_steps < 1) return fail(ENV_EINVAL, "k_steps must be >= 1");
    if (!stream) return fail(ENV_EINVAL, "graph capture needs a non-null stream");
    if (b->plan.G > 0 && (!act || !obs || !reward)) return fail(ENV_EINVAL, "act/obs/reward is NULL");
    hipStream_t s = as_stream(stream);
    int t;
    int rc = batch_prepare(b, s, &t);
    if (rc != ENV_OK) return rc;
    *table = t;
    const int64_t G = b->plan.G;
    // the first step may sort by strips only if every env is in cell order;
    // the steps after it always may
    StepPlan first = b->plan, later = b->plan;
    first.strip_now = batch_sorted(b);
    later.strip_now = 1;
    std::vector<uint64_t> key = {(uint64_t)k_steps, key_of(act), key_of(obs), key_of(reward),
                                 key_of(s), (uint64_t)first.strip_now};
    return capture_graph(b->gc[t], std::move(key), s, [&]() {
        hipError_t le = hipSuccess;
        for (int k = 0; k < k_steps && le == hipSuccess; ++k)
            le = launch_step(k == 0 ? first : later, t ^ (k & 1), 1, act + (size_t)k * G * 2, obs,
                             reward + (size_t)k * G, 1, s);
        return le;
    });
}

int env_batch_capture(env_batch_t *b, int k_steps, const float *act, float *obs, float *reward,
                      void *stream) {
    int t;
    return batch_capture(b, k_steps, act, obs, reward, stream, &t);
}

int env_batch_run(env_batch_t *b, int k_steps, const float *act, float *obs, float *reward,
                  void *stream) {
    int t;
    int rc = batch_capture(b, k_steps, act, obs, reward, stream, &t);
    if (rc != ENV_OK) return rc;
    hipError_t e = hipGraphLaunch(b->gc[t].exec, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    batch_advance(b, k_steps);
    return ENV_OK;
}

}  // extern "C"

// Shared by env_rollout (one policy) and env_rollout_tag (runner and chaser
// policies; log_std then holds the runner's two values, then the chaser's).
static int rollout_impl(env_batch_t *b, pol_t *pol, pol_t *chaser, int steps, const float *log_std,
                        const float *eps, float *obs, float *act, float *logp, float *reward,
                        void *stream) {
    if (!b || !pol) return fail(ENV_EINVAL, "batch or policy is NULL");
    const bool tag = b->plan.tag != 0;
    if (tag != (chaser != nullptr))
        return fail(ENV_EINVAL, tag ? "tag batches need env_rollout_tag (two policies)"
                                    : "env_rollout_tag needs a batch of tag envs");
    for (pol_t *q : {pol, chaser}) {
        if (!q) continue;
        if (policy_is_critic(q)) return fail(ENV_EINVAL, "rollouts need actors, not critics");
        if (policy_in_dim(q) != b->plan.obs_dim)
            return fail(ENV_EINVAL, "policy input %d != observation length %d", policy_in_dim(q),
                        b->plan.obs_dim);
    }
    if (steps < 1) return fail(ENV_EINVAL, "steps must be >= 1");
    if (!stream) return fail(ENV_EINVAL, "rollouts need a non-null stream (graph capture)");
    if (eps && !log_std) return fail(ENV_EINVAL, "sampling (eps) needs log_std");
    if (!eps && logp) return fail(ENV_EINVAL, "logp needs sampling (eps)");
    const int n_ls = tag ? 4 : 2;
    float ls[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k = 0; k < n_ls && log_std; ++k) {
        if (!isfinite(log_std[k])) return fail(ENV_EINVAL, "log_std must be finite");
        ls[k] = log_std[k];
    }
    const int64_t G = b->plan.G;
    if (G > 0 && (!obs || !act || !reward)) return fail(ENV_EINVAL, "obs/act/reward is NULL");
    hipStream_t s = as_stream(stream);
    int t;
    int rc = batch_prepare(b, s, &t);
    if (rc != ENV_OK) return rc;
    const int d = b->plan.obs_dim;
    uint32_t lsb[4];
    memcpy(lsb, ls, sizeof(lsb));
    std::vector<uint64_t> key = {(uint64_t)steps, key_of(policy_weights(pol)),
                                 key_of(chaser ? policy_weights(chaser) : nullptr), key_of(eps),
                                 key_of(obs), key_of(act), key_of(logp), key_of(reward),
                                 key_of(s), ((uint64_t)lsb[0] << 32) | lsb[1],
                                 ((uint64_t)lsb[2] << 32) | lsb[3]};
    const bool fuse_plan = !tag && b->fuse_policy && plan_fuses_policy(b->plan);
    StepPlan first = b->plan, later = b->plan;
    first.strip_now = batch_sorted(b);
    later.strip_now = 1;
    key.push_back((uint64_t)first.strip_now);
    rc = capture_graph(b->rgc[t], std::move(key), s, [&]() {
        hipError_t le = hipSuccess;
        for (int k = 0; k < steps && le == hipSuccess; ++k) {
            const int tk = t ^ (k & 1);
            const float *o_k = obs + (size_t)k * G * d;
            float *a_k = act + (size_t)k * G * 2;
            const float *e_k = eps ? eps + (size_t)k * G * 2 : nullptr;
            float *l_k = logp ? logp + (size_t)k * G : nullptr;
            if (tag) {
                le = policy_launch_typed(pol, b->plan, tk, 0, o_k, e_k, ls, a_k, l_k, s);
                if (le == hipSuccess)
                    le = policy_launch_typed(chaser, b->plan, tk, 1, o_k, e_k, ls + 2, a_k, l_k, s);
            } else if (k == 0 || !fuse_plan) {
                // the first action; when the plan fuses, each step's view
                // sweep then computes the next
                le = eps ? policy_launch_sample(pol, o_k, G, e_k, ls, a_k, l_k, s)
                         : policy_launch(pol, o_k, G, a_k, s);
            }
            PolFuse pf{};
            const bool fuse = fuse_plan && k + 1 < steps;
            if (fuse) {
                pf = policy_fuse_args(pol);
                pf.act = reinterpret_cast<float2 *>(act + (size_t)(k + 1) * G * 2);
                if (eps)
                    policy_fuse_sampling(&pf, ls, eps + (size_t)(k + 1) * G * 2,
                                         logp ? logp + (size_t)(k + 1) * G : nullptr);
            }
            if (le == hipSuccess)
                le = launch_step(k == 0 ? first : later, tk, 1, a_k, obs + (size_t)(k + 1) * G * d,
                                 reward + (size_t)k * G, 1, s, nullptr, fuse ? &pf : nullptr);
        }
        return le;
    });
    if (rc != ENV_OK) return rc;
    hipError_t e = hipGraphLaunch(b->rgc[t].exec, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    batch_advance(b, steps);
    return ENV_OK;
}

extern "C" {

int env_rollout(env_batch_t *b, pol_t *pol, int steps, const float *log_std, const float *eps,
                float *obs, float *act, float *logp, float *reward, void *stream) {
    return rollout_impl(b, pol, nullptr, steps, log_std, eps, obs, act, logp, reward, stream);
}

int env_rollout_tag(env_batch_t *b, pol_t *runner, pol_t *chaser, int steps,
                    const float *log_std, const float *eps, float *obs, float *act, float *logp,
                    float *reward, void *stream) {
    if (!chaser) return fail(ENV_EINVAL, "chaser policy is NULL");
    return rollout_impl(b, runner, chaser, steps, log_std, eps, obs, act, logp, reward, stream);
}

int env_step_policy_tag(env_batch_t *b, pol_t *runner, pol_t *chaser, float *act, float *obs,
                        float *reward, void *stream) {
    if (!b || !runner || !chaser) return fail(ENV_EINVAL, "batch or policy is NULL");
    if (!b->plan.tag) return fail(ENV_EINVAL, "env_step_policy_tag needs a batch of tag envs");
    if (b->plan.G > 0 && (!act || !obs || !reward)) return fail(ENV_EINVAL, "act/obs/reward is NULL");
    for (pol_t *q : {runner, chaser}) {
        if (policy_is_critic(q)) return fail(ENV_EINVAL, "env_step_policy_tag needs actors");
        if (policy_in_dim(q) != b->plan.obs_dim)
            return fail(ENV_EINVAL, "policy input %d != observation length %d", policy_in_dim(q),
                        b->plan.obs_dim);
    }
    hipStream_t s = as_stream(stream);
    int t;
    int rc = batch_prepare(b, s, &t);
    if (rc != ENV_OK) return rc;
    hipError_t e = policy_launch_typed(runner, b->plan, t, 0, obs, nullptr, nullptr, act, nullptr, s);
    if (e == hipSuccess)
        e = policy_launch_typed(chaser, b->plan, t, 1, obs, nullptr, nullptr, act, nullptr, s);
    b->plan.strip_now = batch_sorted(b);
    if (e == hipSuccess) e = launch_step(b->plan, t, 1, act, obs, reward, 1, s);
    if (e != hipSuccess) return hip_fail(e, "env_step_policy_tag");
    batch_advance(b, 1);
    return ENV_OK;
}

int env_step_policy(env_batch_t *b, pol_t *pol, float *act, float *obs, float *reward,
                    void *stream) {
    if (!b || !pol) return fail(ENV_EINVAL, "batch or policy is NULL");
    if (b->plan.G > 0 && (!act || !obs || !reward)) return fail(ENV_EINVAL, "act/obs/reward is NULL");
    if (policy_is_critic(pol)) return fail(ENV_EINVAL, "env_step_policy needs an actor, not a critic");
    if (b->plan.tag) return fail(ENV_EINVAL, "tag batches need env_step_policy_tag (two policies)");
    if (policy_in_dim(pol) != b->plan.obs_dim)
        return fail(ENV_EINVAL, "policy input %d != observation length %d", policy_in_dim(pol),
                    b->plan.obs_dim);
    hipStream_t s = as_stream(stream);
    int t;
    int rc = batch_prepare(b, s, &t);
    if (rc != ENV_OK) return rc;
    if (!b->fuse_policy || !plan_fuses_policy(b->plan)) {
        // the policy as its own launch before the step
        hipError_t e = policy_launch(pol, obs, b->plan.G, act, s);
        b->plan.strip_now = batch_sorted(b);
        if (e == hipSuccess) e = launch_step(b->plan, t, 1, act, obs, reward, 1, s);
        if (e != hipSuccess) return hip_fail(e, "env_step_policy");
        batch_advance(b, 1);
        return ENV_OK;
    }
    bool have_next = b->next_valid && b->next_pol == policy_weights(pol) && b->next_obs == obs;
    for (size_t k = 0; k < b->envs.size() && have_next; ++k)
        have_next = b->envs[k]->gen == b->next_gen[k];
    float *nxt = reinterpret_cast<float *>(b->act_next);
    hipError_t e = hipSuccess;
    if (!have_next) e = policy_launch(pol, obs, b->plan.G, nxt, s);
    // the step applies the actions in act_next (copying them to act) and its
    // view sweep writes the next step's actions there
    PolFuse pf = policy_fuse_args(pol);
    pf.act = b->act_next;
    b->plan.strip_now = batch_sorted(b);
    if (e == hipSuccess) e = launch_step(b->plan, t, 1, nxt, obs, reward, 1, s, nullptr, &pf, act);
    if (e != hipSuccess) {
        b->next_valid = false;
        return hip_fail(e, "env_step_policy");
    }
    batch_advance(b, 1);
    b->next_valid = b->plan.G > 0;
    b->next_pol = policy_weights(pol);
    b->next_obs = obs;
    b->next_gen.resize(b->envs.size());
    for (size_t k = 0; k < b->envs.size(); ++k) b->next_gen[k] = b->envs[k]->gen;
    return ENV_OK;
}

}  // extern "C"
