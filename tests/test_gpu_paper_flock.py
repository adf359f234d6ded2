"""GPU parity for the paper's own flock settings (Sec. 4.1 and 5).

v = 128 sectors over a 250-degree field of view, the agent's speed appended
to its view (129 values per row), vision range one tenth of the box side.
Checks are teacher-forced: the oracle moves the GPU's pre-step state with the
same actions (heading and speed bitwise, positions within the move
tolerance) and senses the GPU's post-move state; the view must lie in the
oracle's bands and the speed column must equal the post-move speed bitwise.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from parity import EPS_D, EPS_PHI, check_move, check_sense

pytestmark = pytest.mark.gpu
flock = pytest.importorskip("paper_2207_03945_amd")

FOV250 = math.radians(250.0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t if isinstance(t, np.ndarray) else t.detach().cpu().numpy()


def params_for(cfg, n=None, **kw):
    p = dict(n_agents=cfg["n"] if n is None else n, box=cfg["box"], radius=cfg["radius"],
             sectors=cfg["sectors"], fov=math.radians(cfg["fov_deg"]),
             flags=flock.ENV_FLAG_COUNTS | (flock.ENV_FLAG_SPEED_OBS if cfg["speed_obs"] else 0))
    p.update(kw)
    return flock.Params(**p)


def oracle_band(st, p, agents=None):
    fov = p.fov if p.fov > 0 else oracle.TWO_PI
    return oracle.oracle_sense(st[0], st[1], st[2], p.box, radius=p.radius, collide=p.collide,
                               sectors=p.sectors, r_nb=p.r_nb, r_col=p.r_col, agents=agents,
                               eps_d=EPS_D, eps_phi=EPS_PHI, fov=fov)


def gpu_state(env):
    return tuple(host(t) for t in env.get_state())


def check_rows(env, pre, act, p, obs, rew, agents=None, label=""):
    """Rows after a step with actions ``act`` from GPU state ``pre`` (act None:
    after the reset of state ``pre``), teacher-forced."""
    torch.cuda.synchronize()
    st = gpu_state(env)
    want = pre if act is None else oracle.oracle_move(pre, act, p.box, p.max_turn, p.max_dspeed,
                                                      p.s_min, p.s_max)
    check_move(st, want, p.box, label)
    rows = slice(None) if agents is None else agents
    o = host(obs)[rows]
    v = p.sectors
    if p.obs_dim > v:
        sp = np.asarray(st[3], np.float32)[rows]
        assert np.array_equal(o[:, v].astype(np.float32), sp), f"{label}: speed column differs"
    nb, col = (host(t) for t in env.counts())
    return check_sense(oracle_band(st, p, agents), o[:, :v], host(rew)[rows], nb[rows], col[rows],
                       radius=p.radius, r_nb=p.r_nb, r_col=p.r_col, label=label)


def run_case(p, st, steps, check_at, n_sample=None, seed=0, label="", lanes=0):
    env = flock.Env(p)
    env.set_state(*[dev(a) for a in st])
    obs0 = env.reset()
    if lanes:
        env.set_sweep_lanes(lanes)
    g = np.random.default_rng(seed + 7)
    n = p.n_agents
    stats = [check_rows(env, st, None, p, obs0, 0.1 * host(env.counts()[0]) - host(env.counts()[1]),
                        label=f"{label} reset")] if n_sample is None else []
    obs = torch.empty(n, p.obs_dim, device="cuda")
    rew = torch.empty(n, device="cuda")
    for t in range(steps):
        act = workloads.random_actions(n, seed=seed, step=t)
        if t in check_at:
            pre = gpu_state(env)
            env.step(dev(act), obs, rew)
            agents = None
            if n_sample is not None:
                agents = np.sort(g.choice(n, size=min(n_sample, n), replace=False)).astype(np.int32)
            stats.append(check_rows(env, pre, act, p, obs, rew, agents, label=f"{label} step {t}"))
        else:
            env.step(dev(act), obs, rew)
    return env, stats


def test_paper_flock1k_every_agent():
    """1,000 agents, box 100, R 10, 128 sectors, FOV 250, speed in the view: all rows, 20 steps."""
    cfg = workloads.WORKLOADS["paper_flock1k"]
    p = params_for(cfg)
    st = workloads.make_state(cfg, seed=0)
    _, stats = run_case(p, st, 20, set(range(20)), label="paper_flock1k")
    print("ambiguous sector cells per step:", [s["ambiguous_sector_cells"] for s in stats])


def test_paper_flock10k_sampled():
    """10,000 agents (about 314 neighbours each), 128 steps; 1,500 sampled rows at five steps."""
    cfg = workloads.WORKLOADS["paper_flock10k"]
    p = params_for(cfg)
    st = workloads.make_state(cfg, seed=1)
    run_case(p, st, cfg["steps"], {0, 1, 2, 50, 127}, n_sample=1500, seed=1, label="paper_flock10k")


@pytest.mark.parametrize("reach,lanes", [(2, 16), (2, 4), (1, 16)])
def test_paper_flock10k_batch_at_timed_settings(reach, lanes):
    """Three 10,000-agent envs batched as the paper-scale leg is timed: cell reach
    2 and 16 lanes per agent (the tuner's choice), and the neighbouring settings;
    500 sampled rows of each env checked at three of six steps."""
    cfg = workloads.WORKLOADS["paper_flock10k"]
    p = params_for(cfg, cell_reach=reach)
    envs, sts = [], []
    for k in range(3):
        st = workloads.make_state(cfg, seed=40 + k)
        e = flock.Env(p)
        e.set_state(*[dev(a) for a in st])
        e.reset()
        envs.append(e)
        sts.append(st)
    assert envs[0].geometry()[2] == reach
    b = flock.Batch(envs)
    b.set_sweep_lanes(lanes)
    G, off, n = b.n, b.offsets, p.n_agents
    obs = torch.empty(G, p.obs_dim, device="cuda")
    rew = torch.empty(G, device="cuda")
    g = np.random.default_rng(reach * 100 + lanes)
    for t in range(6):
        act = workloads.random_actions(G, seed=41, step=t)
        pre = [gpu_state(e) for e in envs]
        b.step(dev(act), obs, rew)
        if t in (0, 2, 5):
            for k in range(3):
                agents = np.sort(g.choice(n, 500, replace=False)).astype(np.int32)
                rows = slice(off[k], off[k + 1])
                check_rows(envs[k], pre[k], act[off[k]:off[k + 1]], p, obs[rows], rew[rows], agents,
                           label=f"env {k} step {t} reach {reach} lanes {lanes}")


@pytest.mark.parametrize("v", [1, 2, 7, 16, 129])
@pytest.mark.parametrize("fov_deg", [30.0, 250.0, 359.0])
def test_fov_sector_counts(v, fov_deg):
    cfg = workloads.WORKLOADS["paper_flock1k"]
    p = params_for(cfg, n=400, sectors=v, fov=math.radians(fov_deg))
    st = workloads.make_state({**cfg, "n": 400}, seed=v)
    run_case(p, st, 3, {0, 2}, seed=v, label=f"v={v} fov={fov_deg}")


@pytest.mark.parametrize("speed_obs", [False, True])
def test_limited_view_without_speed_and_full_view_with_speed(speed_obs):
    cfg = workloads.WORKLOADS["paper_flock1k"]
    kw = dict(flags=flock.ENV_FLAG_COUNTS | (flock.ENV_FLAG_SPEED_OBS if speed_obs else 0))
    kw["fov"] = 0.0 if speed_obs else FOV250
    p = params_for(cfg, n=600, **kw)
    st = workloads.make_state({**cfg, "n": 600}, seed=3)
    run_case(p, st, 4, {0, 3}, seed=3, label=f"speed_obs={speed_obs}")


def test_coincident_agents_seen_straight_ahead():
    """Coincident agents lie on the heading: middle sector v/2 under a limited view."""
    v, box = 16, 100.0
    x = np.array([50.0, 50.0, 10.0], np.float32)
    y = np.array([50.0, 50.0, 10.0], np.float32)
    th = np.array([0.3, 2.0, 0.0], np.float32)
    s = np.ones(3, np.float32)
    p = flock.Params(n_agents=3, box=box, radius=10.0, sectors=v, fov=FOV250,
                     flags=flock.ENV_FLAG_COUNTS)
    env = flock.Env(p)
    env.set_state(*[dev(a) for a in (x, y, th, s)])
    obs = host(env.reset())
    torch.cuda.synchronize()
    for i in (0, 1):
        assert obs[i, v // 2] == 1.0 and np.count_nonzero(obs[i]) == 1, obs[i]
    assert not obs[2].any()
    nb, col = env.counts()
    check_rows(env, (x, y, th, s), None, p, torch.from_numpy(obs), 0.1 * nb.float() - col.float(),
               label="coincident")


def test_batch_mixing_views_equals_plain_bitwise():
    """A batch of full- and limited-view envs gives the same bits as each env alone."""
    cfg = workloads.WORKLOADS["paper_flock1k"]
    sizes = [300, 1000, 37, 512]
    fovs = [FOV250, 0.0, math.radians(90.0), FOV250]
    ps = [params_for(cfg, n=n, fov=f) for n, f in zip(sizes, fovs)]
    sts = [workloads.make_state({**cfg, "n": n}, seed=10, env=k) for k, n in enumerate(sizes)]
    plain, batched = [], []
    for p, st in zip(ps, sts):
        for lst in (plain, batched):
            e = flock.Env(p)
            e.set_state(*[dev(a) for a in st])
            e.reset()
            lst.append(e)
    b = flock.Batch(batched)
    G, d = b.n, b.d
    assert d == 129
    obs_b = torch.empty(G, d, device="cuda")
    rew_b = torch.empty(G, device="cuda")
    for t in range(5):
        act = workloads.random_actions(G, seed=10, step=t)
        b.step(dev(act), obs_b, rew_b)
        for k, e in enumerate(plain):
            lo, hi = b.offsets[k], b.offsets[k + 1]
            o, r = e.step(dev(act[lo:hi]))
            assert torch.equal(o, obs_b[lo:hi]) and torch.equal(r, rew_b[lo:hi]), (t, k)


def test_graph_run_limited_view_matches_eager():
    cfg = workloads.WORKLOADS["paper_flock1k"]
    p = params_for(cfg)
    st = workloads.make_state(cfg, seed=4)
    envs = []
    for _ in range(2):
        e = flock.Env(p)
        e.set_state(*[dev(a) for a in st])
        e.reset()
        envs.append(e)
    b_graph, b_eager = flock.Batch([envs[0]]), flock.Batch([envs[1]])
    k = 6
    n, d = p.n_agents, p.obs_dim
    act = dev(np.stack([workloads.random_actions(n, seed=4, step=t) for t in range(k)]))
    obs_g = torch.empty(n, d, device="cuda")
    rew_g = torch.empty(k, n, device="cuda")
    stream = torch.cuda.Stream()
    for rep in range(2):
        with torch.cuda.stream(stream):
            b_graph.run(k, act, obs_g, rew_g, stream)
        stream.synchronize()
        obs_e = torch.empty(n, d, device="cuda")
        for t in range(k):
            rew_e = torch.empty(n, device="cuda")
            b_eager.step(act[t].contiguous(), obs_e, rew_e)
            assert torch.equal(rew_e, rew_g[t]), (rep, t)
        torch.cuda.synchronize()
        assert torch.equal(obs_e, obs_g), rep


def test_policy_drives_speed_obs_env():
    """env_step_policy with a 129-input policy equals forward + step."""
    cfg = workloads.WORKLOADS["paper_flock1k"]
    p = params_for(cfg)
    st = workloads.make_state(cfg, seed=5)
    ws, bs = workloads.xavier_weights([p.obs_dim, 64, 64, 2], seed=5)
    pol = flock.Policy(ws, bs)
    envs = []
    for _ in range(2):
        e = flock.Env(p)
        e.set_state(*[dev(a) for a in st])
        envs.append(e)
    obs_a = envs[0].reset()
    obs_b = envs[1].reset()
    ba, bb = flock.Batch([envs[0]]), flock.Batch([envs[1]])
    n = p.n_agents
    act_a = torch.empty(n, 2, device="cuda")
    rew_a = torch.empty(n, device="cuda")
    rew_b = torch.empty(n, device="cuda")
    for t in range(4):
        ba.step_policy(pol, act_a, obs_a, rew_a)
        act_b = pol.forward(obs_b)
        bb.step(act_b, obs_b, rew_b)
        torch.cuda.synchronize()
        assert torch.equal(act_a, act_b) and torch.equal(obs_a, obs_b) and torch.equal(rew_a, rew_b), t
