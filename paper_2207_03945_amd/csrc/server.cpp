// server.cpp -- continuous-batching episode server over the batched step.
//
// Episode requests (an env's parameters, its initial state and an episode
// length) arrive at any time.  Each tick admits queued requests whose device
// memory fits in the caller's arena, then runs ONE closed-loop batched step
// (shared policy -> actions -> move -> view/reward -> FP64 returns) over every
// running request, and retires the requests that reached their length.  State
// stays resident on the device for the whole episode (Sec. 2.2 of
// arXiv:2207.03945: environment and learner exchange data on the device, with
// no copy through the host); only the initial state goes up and the final
// FP64 returns come down.
//
// Memory: each running request owns two arena blocks (its env workspace and
// its act/obs/reward rows); the batch sort scratch is one more block, resized
// whenever the running set changes.  A request is admitted only when its
// blocks AND the resized scratch fit, so a running set can always step.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <vector>

#include "flock_internal.h"

using namespace flock;

namespace {

// First-fit allocator of 256-byte-aligned blocks inside [0, size).
class ArenaAlloc {
public:
    explicit ArenaAlloc(size_t size = 0) { reset(size); }
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align_up(bytes ? bytes : 1, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes ? bytes : 1, 256);
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

struct Block {
    size_t off = 0, bytes = 0;
    bool live = false;
};

struct Request {
    int64_t id = 0;
    env_params_t p{};
    int steps = 0, done = 0;
    int state = 0;  // 0 queued, 1 running, 2 finished
    int head_ticks = 0;  // ticks spent at the head of the queue without being admitted
    std::vector<float> x, y, th, s;
    std::vector<double> ret;
    env_t *env = nullptr;
    Block ws, io;
    float *act = nullptr, *obs = nullptr, *rew = nullptr;
};

size_t io_bytes(const env_params_t &p) {
    const size_t n = (size_t)p.n_agents;
    return align_up(n * 2 * sizeof(float), 256) + align_up(n * obs_dim_of(p) * sizeof(float), 256) +
           align_up(n * sizeof(float), 256);
}

}  // namespace

struct flock_server {
    char *arena = nullptr;
    size_t arena_bytes = 0;
    int max_slots = 0;
    int layout_v = 0;             // sectors of every request (0 until the first submit)
    pol_t *pol = nullptr;
    hipStream_t stream = nullptr;
    ArenaAlloc alloc;
    Block scratch;
    StepPlan plan{};
    std::vector<DevEnv> tab[2];   // [t]: each running env oriented for tick parity t
    std::vector<int32_t> base;
    int table = 0;                // table of the next tick
    bool dirty = true;
    std::deque<int64_t> queue;
    std::map<int64_t, Request> reqs;
    std::vector<int64_t> running;
    int64_t next_id = 1;
};

namespace {

int64_t running_agents(const srv_t *S, int64_t *cells) {
    int64_t g = 0, c = 0;
    for (int64_t id : S->running) {
        const Request &r = S->reqs.at(id);
        g += r.p.n_agents;
        c += env_cell_count(r.env);
    }
    *cells = c;
    return g;
}

// Columns of an env's grid: at most one strip each, so a bound on the strips
// of any plan that holds the env.
int64_t env_columns(const env_t *env) { return env_descriptor(env, 0).ncx; }

int64_t running_columns(const srv_t *S) {
    int64_t c = 0;
    for (int64_t id : S->running) c += env_columns(S->reqs.at(id).env);
    return c;
}

// (Re)allocate the sort scratch for G agents / C cells / E envs; restores the
// previous block on failure.
bool resize_scratch(srv_t *S, int64_t G, int64_t C, int E, int64_t cols) {
    const Block old = S->scratch;
    if (old.live) S->alloc.release(old.off, old.bytes);
    Block nb;
    nb.bytes = sort_scratch_bytes(G, C, E > 0 ? E : 1, cols);
    if (S->alloc.alloc(nb.bytes, &nb.off)) {
        nb.live = true;
        S->scratch = nb;
        S->dirty = true;
        return true;
    }
    if (old.live) {
        size_t off = 0;
        S->alloc.alloc(old.bytes, &off);  // the block just released is free again
        S->scratch = old;
        S->scratch.off = off;
        S->dirty = true;                  // it may have moved: rebuild the tables
    }
    return false;
}

void release_request_blocks(srv_t *S, Request &r) {
    if (r.env) {
        env_destroy(r.env);
        r.env = nullptr;
    }
    if (r.ws.live) S->alloc.release(r.ws.off, r.ws.bytes);
    if (r.io.live) S->alloc.release(r.io.off, r.io.bytes);
    r.ws.live = r.io.live = false;
}

// Try to place a queued request on the device.  ENV_OK, ENV_EAGAIN or an error.
int try_admit(srv_t *S, Request &r) {
    if ((int)S->running.size() >= S->max_slots) return ENV_EAGAIN;
    r.ws.bytes = env_workspace_bytes(&r.p);
    r.io.bytes = io_bytes(r.p);
    if (!S->alloc.alloc(r.ws.bytes, &r.ws.off)) return ENV_EAGAIN;
    r.ws.live = true;
    if (!S->alloc.alloc(r.io.bytes, &r.io.off)) {
        release_request_blocks(S, r);
        return ENV_EAGAIN;
    }
    r.io.live = true;
    int rc = env_create(&r.p, S->arena + r.ws.off, r.ws.bytes, &r.env);
    if (rc != ENV_OK) {
        release_request_blocks(S, r);
        return rc;
    }
    int64_t C;
    const int64_t G = running_agents(S, &C);
    if (!resize_scratch(S, G + r.p.n_agents, C + env_cell_count(r.env), (int)S->running.size() + 1,
                        running_columns(S) + env_columns(r.env))) {
        release_request_blocks(S, r);
        return ENV_EAGAIN;
    }
    const size_t n = (size_t)r.p.n_agents;
    char *io = S->arena + r.io.off;
    r.act = reinterpret_cast<float *>(io);
    r.obs = reinterpret_cast<float *>(io + align_up(n * 2 * sizeof(float), 256));
    r.rew = reinterpret_cast<float *>(io + align_up(n * 2 * sizeof(float), 256) +
                                      align_up(n * obs_dim_of(r.p) * sizeof(float), 256));
    rc = env_load_host_state(r.env, r.x.data(), r.y.data(), r.th.data(), r.s.data(), S->stream);
    if (rc == ENV_OK) rc = env_reset(r.env, r.obs, S->stream);
    if (rc != ENV_OK) {
        release_request_blocks(S, r);
        return rc;
    }
    r.state = 1;
    S->running.push_back(r.id);
    S->dirty = true;
    return ENV_OK;
}

// Ticks the head of the queue may be passed over by later requests that fit
// before admission stops at it until it fits (it always fits eventually:
// running requests finish in a bounded number of ticks and srv_submit
// rejects requests larger than the arena).
constexpr int kHeadPatience = 32;

void admit_queued(srv_t *S) {
    for (auto it = S->queue.begin(); it != S->queue.end();) {
        Request &r = S->reqs.at(*it);
        if (try_admit(S, r) == ENV_OK) {
            it = S->queue.erase(it);
            continue;
        }
        if (it == S->queue.begin() && ++r.head_ticks > kHeadPatience) break;  // hold for the head
        ++it;
    }
}

int rebuild_plan(srv_t *S) {
    for (auto &t : S->tab) t.clear();
    S->base.clear();
    int64_t g = 0, c = 0;
    for (int64_t id : S->running) {
        Request &r = S->reqs.at(id);
        for (int f = 0; f < 2; ++f) {
            DevEnv d = env_descriptor(r.env, f);
            d.agent_base = (int32_t)g;
            d.cell_base = (int32_t)c;
            d.act = r.act;
            d.obs = r.obs;
            d.rew = r.rew;
            S->tab[f].push_back(d);
        }
        S->base.push_back((int32_t)g);
        g += r.p.n_agents;
        c += env_cell_count(r.env);
    }
    S->base.push_back((int32_t)g);
    // strips of the running envs (the strip sort), when every env allows it
    bool strips_ok = true;
    for (const DevEnv &d : S->tab[0]) strips_ok = strips_ok && strips_allowed(d);
    std::vector<int32_t> strip_env;
    int64_t n_strips = 0;
    if (strips_ok && !S->tab[0].empty()) {
        DevEnv *tabs[2] = {S->tab[0].data(), S->tab[1].data()};
        n_strips = assign_strips(tabs, 2, (int)S->running.size(), g, &strip_env);
    }
    Carver cv{S->arena + S->scratch.off, 0};
    carve_sort(cv, g, c, (int)S->running.size(), &S->plan.a, n_strips);
    S->plan.strips = (int)n_strips;
    if (n_strips > 0) plan_strip_launch(&S->plan, S->tab[0].data(), (int)S->running.size());
    S->plan.n_envs = (int)S->running.size();
    S->plan.G = g;
    S->plan.C = c;
    S->plan.v = S->running.empty() ? 1 : S->reqs.at(S->running[0]).p.sectors;
    S->plan.obs_dim = S->running.empty() ? 1 : obs_dim_of(S->reqs.at(S->running[0]).p);
    S->plan.fov = 0;
    double cand = 0.0;
    for (int64_t rid : S->running) {
        const Request &r = S->reqs.at(rid);
        if (!full_view(r.p)) S->plan.fov = 1;
        cand += env_candidates_per_agent(r.env) * r.p.n_agents;
    }
    S->plan.lanes = auto_lanes(g > 0 ? cand / (double)g : 0.0, S->plan.v, (int64_t)g);
    int64_t max_cells = 0, max_agents = 0;
    for (int64_t rid : S->running) {
        max_cells = std::max(max_cells, env_cell_count(S->reqs.at(rid).env));
        max_agents = std::max(max_agents, (int64_t)S->reqs.at(rid).p.n_agents);
    }
    S->plan.max_env_cells = max_cells;
    S->plan.env_sort_recs = env_sort_recs_for((int)S->running.size(), max_agents, max_cells);
    S->plan.scan_blocks = scan_blocks_for(c, max_cells);
    hipError_t e = hipSuccess;
    for (int f = 0; f < 2 && e == hipSuccess; ++f)
        e = hipMemcpyAsync(S->plan.a.envs[f], S->tab[f].data(), S->tab[f].size() * sizeof(DevEnv),
                           hipMemcpyHostToDevice, S->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->plan.a.base, S->base.data(), S->base.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, S->stream);
    if (e == hipSuccess && n_strips > 0)
        e = hipMemcpyAsync(S->plan.a.strip_env, strip_env.data(), strip_env.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, S->stream);
    if (e == hipSuccess) e = launch_clear(S->plan, S->stream);
    if (e != hipSuccess) return set_error(ENV_EHIP, "serving plan upload: %s", hipGetErrorString(e));
    S->table = 0;
    S->dirty = false;
    return ENV_OK;
}

}  // namespace

extern "C" {

size_t srv_request_bytes(const env_params_t *p) {
    if (validate_params(p) != ENV_OK) return 0;
    const size_t ws = align_up(env_workspace_bytes(p), 256);
    // its share of the batch sort scratch: per agent and per cell arrays
    const int64_t n = p->n_agents;
    const size_t share = sort_scratch_bytes(n, cell_count_for(*p), 1, column_count_for(*p));
    return ws + io_bytes(*p) + share;
}

int srv_create(void *arena, size_t arena_bytes, int max_slots, pol_t *pol, void *stream,
               srv_t **out) {
    if (!arena || !pol || !out) return set_error(ENV_EINVAL, "NULL argument to srv_create");
    if (reinterpret_cast<uintptr_t>(arena) % 256 != 0)
        return set_error(ENV_EINVAL, "arena must be 256-byte aligned");
    if (max_slots < 1) return set_error(ENV_EINVAL, "max_slots must be >= 1");
    if (policy_is_critic(pol)) return set_error(ENV_EINVAL, "the server needs an actor, not a critic");
    srv_t *S = new srv_t;
    S->arena = static_cast<char *>(arena);
    S->arena_bytes = arena_bytes;
    S->max_slots = max_slots;
    S->pol = pol;
    S->stream = reinterpret_cast<hipStream_t>(stream);
    S->alloc.reset(arena_bytes);
    *out = S;
    return ENV_OK;
}

void srv_destroy(srv_t *S) {
    if (!S) return;
    for (auto &kv : S->reqs)
        if (kv.second.env) env_destroy(kv.second.env);
    delete S;
}

int srv_submit(srv_t *S, const env_params_t *p, const float *x, const float *y, const float *th,
               const float *s, int steps, int64_t *id) {
    if (!S || !id) return set_error(ENV_EINVAL, "NULL argument to srv_submit");
    int rc = validate_params(p);
    if (rc != ENV_OK) return rc;
    if (p->flags & ENV_FLAG_TAG)
        return set_error(ENV_EINVAL, "the server runs flock requests (one shared policy), not tag");
    if (obs_dim_of(*p) != policy_in_dim(S->pol))
        return set_error(ENV_EINVAL, "request observations have %d values, policy takes %d",
                         obs_dim_of(*p), policy_in_dim(S->pol));
    // Every request of a server shares one view layout: the first accepted fixes it.
    if (S->layout_v != 0 && p->sectors != S->layout_v)
        return set_error(ENV_EINVAL, "request has %d sectors, this server serves %d",
                         p->sectors, S->layout_v);
    if (steps < 1) return set_error(ENV_EINVAL, "steps must be >= 1");
    const size_t n = (size_t)p->n_agents;
    if (n > 0 && (!x || !y || !th || !s)) return set_error(ENV_EINVAL, "state pointer is NULL");
    const size_t need = srv_request_bytes(p);
    if (need > S->arena_bytes)
        return set_error(ENV_ENOMEM, "request needs %zu bytes, arena has %zu", need, S->arena_bytes);
    S->layout_v = p->sectors;
    Request r;
    r.id = S->next_id++;
    r.p = *p;
    r.steps = steps;
    r.x.assign(x, x + n);
    r.y.assign(y, y + n);
    r.th.assign(th, th + n);
    r.s.assign(s, s + n);
    *id = r.id;
    S->reqs.emplace(r.id, std::move(r));
    Request &rr = S->reqs.at(*id);
    if (S->queue.empty()) {
        rc = try_admit(S, rr);
        if (rc == ENV_OK) return ENV_OK;
        if (rc != ENV_EAGAIN) {
            S->reqs.erase(*id);
            return rc;
        }
    }
    S->queue.push_back(*id);
    set_error(ENV_EAGAIN, "request %lld queued", (long long)*id);
    return ENV_EAGAIN;
}

int srv_tick(srv_t *S, int32_t *n_running, int64_t *agents) {
    if (!S) return set_error(ENV_EINVAL, "server is NULL");
    admit_queued(S);
    if (n_running) *n_running = (int32_t)S->running.size();
    if (agents) *agents = 0;
    if (S->running.empty()) return ENV_OK;
    int rc = ENV_OK;
    if (S->dirty) rc = rebuild_plan(S);
    if (rc != ENV_OK) return rc;
    // the policy on every running request's view (its own launch: run inside
    // the view sweep it was measured slower), then one batched step
    bool sorted = true;  // every running env's records in cell order (after its reset)
    for (int64_t id : S->running) sorted = sorted && env_sorted(S->reqs.at(id).env);
    S->plan.strip_now = sorted ? 1 : 0;
    hipError_t e = policy_launch_envs(S->pol, S->plan, S->table, S->stream);
    if (e == hipSuccess)
        e = launch_step(S->plan, S->table, 1, nullptr, nullptr, nullptr, 1, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) return set_error(ENV_EHIP, "srv_tick: %s", hipGetErrorString(e));
    for (int64_t id : S->running) env_advance(S->reqs.at(id).env, 1);
    S->table ^= 1;
    if (agents) *agents = S->plan.G;
    std::vector<int64_t> still;
    bool changed = false;
    for (int64_t id : S->running) {
        Request &r = S->reqs.at(id);
        r.done += 1;
        if (r.done < r.steps) {
            still.push_back(id);
            continue;
        }
        r.ret.assign(r.p.n_agents, 0.0);
        if (r.p.n_agents > 0) {
            // returns and agent ids of the current (cell-order) buffer
            const DevEnv d = env_descriptor(r.env, 0);
            std::vector<double> ret_cell(r.p.n_agents);
            std::vector<int32_t> id_cell(r.p.n_agents);
            e = hipMemcpy(ret_cell.data(), d.ret_cur, ret_cell.size() * sizeof(double),
                          hipMemcpyDeviceToHost);
            if (e == hipSuccess)
                e = hipMemcpy(id_cell.data(), d.id_cur, id_cell.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost);
            if (e != hipSuccess) return set_error(ENV_EHIP, "returns download: %s", hipGetErrorString(e));
            for (size_t p = 0; p < id_cell.size(); ++p) r.ret[id_cell[p]] = ret_cell[p];
        }
        r.state = 2;
        release_request_blocks(S, r);
        std::vector<float>().swap(r.x);
        std::vector<float>().swap(r.y);
        std::vector<float>().swap(r.th);
        std::vector<float>().swap(r.s);
        changed = true;
    }
    S->running.swap(still);
    if (changed) {
        int64_t C;
        const int64_t G = running_agents(S, &C);
        if (!S->running.empty()) {
            resize_scratch(S, G, C, (int)S->running.size(), running_columns(S));
        } else if (S->scratch.live) {  // an idle server holds no scratch: the arena is whole
            S->alloc.release(S->scratch.off, S->scratch.bytes);
            S->scratch.live = false;
        }
        S->dirty = true;
    }
    return ENV_OK;
}

int srv_poll(srv_t *S, int64_t id, int32_t *state, int32_t *steps_done) {
    if (!S) return set_error(ENV_EINVAL, "server is NULL");
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return set_error(ENV_ENOTFOUND, "unknown request %lld", (long long)id);
    if (state) *state = it->second.state;
    if (steps_done) *steps_done = it->second.done;
    return ENV_OK;
}

int srv_result(srv_t *S, int64_t id, double *returns_host, int64_t n) {
    if (!S) return set_error(ENV_EINVAL, "server is NULL");
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return set_error(ENV_ENOTFOUND, "unknown request %lld", (long long)id);
    Request &r = it->second;
    if (r.state != 2) return set_error(ENV_ESTATE, "request %lld not finished", (long long)id);
    if (n != (int64_t)r.ret.size()) return set_error(ENV_EINVAL, "n = %lld, request has %zu agents",
                                                     (long long)n, r.ret.size());
    if (n > 0 && !returns_host) return set_error(ENV_EINVAL, "returns_host is NULL");
    if (n > 0) memcpy(returns_host, r.ret.data(), n * sizeof(double));
    S->reqs.erase(it);
    return ENV_OK;
}

}  // extern "C"
