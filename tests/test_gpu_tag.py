"""GPU tag environment (Sec. 4.2: runners and chasers) against the oracle.

Teacher-forced: the oracle moves the GPU's pre-step state with the same
actions (heading and speed bitwise, positions within the move tolerance of
``tests/parity.py``) and senses the GPU's post-move state; near/touch counts
must lie in the oracle's bands; each view channel within the bands; rewards
follow the counts by type.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from parity import EPS_D, EPS_PHI, REW_TOL, check_move, check_sense

pytestmark = pytest.mark.gpu
flock = pytest.importorskip("paper_2207_03945_amd")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t if isinstance(t, np.ndarray) else t.detach().cpu().numpy()


def params(cfg, n=None, chasers=None, **kw):
    p = dict(n_agents=cfg["n"] if n is None else n, box=cfg["box"], radius=cfg["radius"],
             collide=cfg["touch"], sectors=cfg["sectors"], fov=math.radians(cfg["fov_deg"]),
             flags=flock.ENV_FLAG_COUNTS | flock.ENV_FLAG_TAG,
             n_chasers=cfg["chasers"] if chasers is None else chasers, r_nb=0.1, r_col=-1.0,
             r_catch=1.0)
    p.update(kw)
    return flock.Params(**p)


def band(st, p, agents=None):
    return oracle.oracle_sense_tag(st[0], st[1], st[2], p.box, p.n_chasers, radius=p.radius,
                                   touch=p.collide, sectors=p.sectors, r_near=p.r_nb,
                                   r_caught=p.r_col, r_catch=p.r_catch, agents=agents,
                                   eps_d=EPS_D, eps_phi=EPS_PHI,
                                   fov=p.fov if p.fov > 0 else oracle.TWO_PI)


def gpu_state(env):
    return tuple(host(t) for t in env.get_state())


def check(env, pre, act, p, obs, rew, agents=None, label=""):
    """The step just taken with ``act`` from GPU state ``pre``, teacher-forced."""
    torch.cuda.synchronize()
    st = gpu_state(env)
    check_move(st, oracle.oracle_move_tag(pre, act, p.box, p.max_turn, p.s_max), p.box, label)
    rows = np.arange(p.n_agents) if agents is None else agents
    o = band(st, p, agents)
    nb, col = (host(t)[rows] for t in env.counts())
    assert ((nb >= o.nb_lo) & (nb <= o.nb_hi)).all(), f"{label}: near counts"
    assert ((col >= o.col_lo) & (col <= o.col_hi)).all(), f"{label}: touch counts"
    r = host(rew)[rows].astype(np.float64)
    chaser = rows < p.n_chasers
    want = np.where(chaser, p.r_catch * col, p.r_nb * nb + p.r_col * col)
    assert (np.abs(r - want) <= REW_TOL * np.maximum(1, np.abs(want))).all(), f"{label}: reward"
    ob = host(obs)[rows]
    check_sense(o, ob[:, :2 * p.sectors], r, None, None, radius=p.radius, label=label)
    if p.obs_dim > 2 * p.sectors:
        assert np.array_equal(ob[:, -1], st[3][rows])
    return int((chaser & (col > 0)).sum())


def run(p, st, steps, check_at, sample=None, lanes=0, seed=0, label=""):
    env = flock.Env(p)
    env.set_sweep_lanes(lanes)
    env.set_state(*[dev(a) for a in st])
    env.reset()
    obs = torch.empty(p.n_agents, p.obs_dim, device="cuda")
    rew = torch.empty(p.n_agents, device="cuda")
    g = np.random.default_rng(seed)
    catches = 0
    for t in range(steps):
        act = workloads.tag_actions(p.n_agents, seed=seed, step=t, s_max=p.s_max)
        pre = gpu_state(env) if t in check_at else None
        env.step(dev(act), obs, rew)
        if t in check_at:
            agents = None if sample is None else np.sort(
                g.choice(p.n_agents, sample, replace=False)).astype(np.int32)
            catches += check(env, pre, act, p, obs, rew, agents, f"{label} step {t}")
    return env, obs, rew, catches


def test_tag_1k_every_agent():
    cfg = workloads.WORKLOADS["paper_tag1k"]
    p = params(cfg)
    st = workloads.make_state(cfg, seed=0)
    _, _, _, catches = run(p, st, 12, set(range(12)), label="tag1k")
    assert catches > 0, "no chaser touched a runner: the touch path went untested"


@pytest.mark.parametrize("reach,lanes", [(0, 1), (0, 16), (2, 16)])
def test_tag_11k_sampled(reach, lanes):
    """11,000 agents (1,000 chasers), 40 steps; reach 2 with 16 lanes per agent is
    the setting the paper-scale tag leg is timed at."""
    cfg = workloads.WORKLOADS["paper_tag11k"]
    p = params(cfg, cell_reach=reach)
    st = workloads.make_state(cfg, seed=1)
    env, *_ = run(p, st, 40, {0, 1, 39}, sample=1500, lanes=lanes, seed=1,
                  label=f"tag11k reach {reach} lanes {lanes}")
    assert reach == 0 or env.geometry()[2] == reach


@pytest.mark.parametrize("speed,full", [(True, False), (False, True)])
def test_tag_speed_column_and_full_view(speed, full):
    cfg = workloads.WORKLOADS["paper_tag1k"]
    kw = {}
    if speed:
        kw["flags"] = flock.ENV_FLAG_COUNTS | flock.ENV_FLAG_TAG | flock.ENV_FLAG_SPEED_OBS
    if full:
        kw["fov"] = 0.0
    p = params(cfg, n=500, chasers=45, **kw)
    st = workloads.make_state({**cfg, "n": 500}, seed=2)
    run(p, st, 4, {0, 3}, seed=2, label=f"speed={speed} full={full}")


@pytest.mark.parametrize("sectors,full", [(8, False), (16, True), (32, False)])
def test_tag_few_sectors_one_lane(sectors, full):
    """One lane per agent with two channels of 8, 16 or 32 sectors (rows of 16,
    32 or 64 values, written whole by the wave), on 700 agents: every agent
    against the oracle over five steps; the last wave of the launch is only
    partly filled."""
    cfg = workloads.WORKLOADS["paper_tag1k"]
    kw = {"sectors": sectors}
    if full:
        kw["fov"] = 0.0
    p = params(cfg, n=700, chasers=64, **kw)
    st = workloads.make_state({**cfg, "n": 700}, seed=5)
    run(p, st, 5, set(range(5)), lanes=1, seed=5, label=f"tag sectors {sectors}")


def test_tag_batch_equals_plain_and_two_policies():
    cfg = workloads.WORKLOADS["paper_tag1k"]
    sizes, chasers = [1100, 300, 12], [100, 27, 1]
    ps = [params(cfg, n=n, chasers=c) for n, c in zip(sizes, chasers)]
    sts = [workloads.make_state({**cfg, "n": n}, seed=5, env=k) for k, n in enumerate(sizes)]

    def envs():
        out = []
        for p, st in zip(ps, sts):
            e = flock.Env(p)
            e.set_state(*[dev(a) for a in st])
            out.append(e)
        return out

    ea, eb = envs(), envs()
    obs_a = torch.cat([e.reset() for e in ea])
    obs_b = torch.cat([e.reset() for e in eb])
    b = flock.Batch(eb)
    d = b.d
    wr, br_ = workloads.xavier_weights([d, 64, 64, 2], seed=1)
    wc, bc = workloads.xavier_weights([d, 64, 64, 2], seed=2)
    runner, chaser = flock.Policy(wr, br_), flock.Policy(wc, bc)
    off = b.offsets
    is_chaser = np.concatenate([np.arange(n) < c for n, c in zip(sizes, chasers)])
    sel = torch.from_numpy(is_chaser).cuda()[:, None]
    act_b = torch.empty(b.n, 2, device="cuda")
    rew_b = torch.empty(b.n, device="cuda")
    for t in range(4):
        b.step_policy_tag(runner, chaser, act_b, obs_b, rew_b)
        want = torch.where(sel, chaser.forward(obs_a), runner.forward(obs_a))
        assert torch.equal(act_b, want), t
        for k, e in enumerate(ea):
            o, r = e.step(want[off[k]:off[k + 1]].contiguous())
            assert torch.equal(o, obs_b[off[k]:off[k + 1]]), (t, k)
            assert torch.equal(r, rew_b[off[k]:off[k + 1]]), (t, k)
        obs_a = torch.cat([obs_b[off[k]:off[k + 1]] for k in range(len(ea))])

    # sampled two-policy rollout equals the same steps one call at a time
    T = 5
    eps = dev(workloads.policy_noise(T, b.n, seed=9))
    ls = (-1.5, -2.0, -1.0, -2.5)
    obs_buf = torch.empty(T + 1, b.n, d, device="cuda")
    act_buf = torch.empty(T, b.n, 2, device="cuda")
    logp_buf = torch.empty(T, b.n, device="cuda")
    rew_buf = torch.empty(T, b.n, device="cuda")
    obs_buf[0].copy_(obs_b)
    obs_s = obs_b.clone()
    b2 = flock.Batch(ea)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.rollout_tag(runner, chaser, T, obs_buf, act_buf, rew_buf, logp=logp_buf, eps=eps,
                      log_std=ls, stream=stream)
    stream.synchronize()
    rew_s = torch.empty(b.n, device="cuda")
    for t in range(T):
        a_r, l_r = runner.sample(obs_s, eps[t].contiguous(), ls[:2])
        a_c, l_c = chaser.sample(obs_s, eps[t].contiguous(), ls[2:])
        act = torch.where(sel, a_c, a_r)
        logp = torch.where(sel[:, 0], l_c, l_r)
        b2.step(act, obs_s, rew_s)
        torch.cuda.synchronize()
        assert torch.equal(act, act_buf[t]) and torch.equal(logp, logp_buf[t]), t
        assert torch.equal(obs_s, obs_buf[t + 1]) and torch.equal(rew_s, rew_buf[t]), t
