"""GPU parity: the HIP step against the CPU oracle, through the C ABI.

Every case draws seeded synthetic inputs from ``workloads``.  Checks are
teacher-forced: the oracle moves the GPU's own pre-step state with the same
actions (heading and speed must match bitwise, positions within the move
tolerance of ``tests/parity.py``), and senses the GPU's post-move state
(counts, view and reward within the bands of ``tests/parity.py``).
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
    return t.detach().cpu().numpy()


def make_env(state, box, v, reach=0, flags=1):
    n = state[0].shape[0]
    env = flock.Env(flock.Params(n_agents=n, box=box, sectors=v, flags=flags, cell_reach=reach))
    env.set_state(*[dev(a) for a in state])
    obs0 = env.reset()
    return env, obs0


def band(state, box, v, agents=None):
    return oracle.oracle_sense(state[0], state[1], state[2], box, sectors=v, agents=agents,
                               eps_d=EPS_D, eps_phi=EPS_PHI)


def gpu_state(env):
    return tuple(host(t) for t in env.get_state())


def check_post(env, pre, act, box, v, obs, rew, agents=None, label=""):
    """Teacher-forced check of the step just taken from GPU state ``pre``."""
    torch.cuda.synchronize()
    post = gpu_state(env)
    check_move(post, oracle.oracle_move(pre, act, box), box, label)
    nb, col = (host(t) for t in env.counts())
    o = band(post, box, v, agents)
    rows = slice(None) if agents is None else agents
    return check_sense(o, host(obs)[rows], host(rew)[rows], nb[rows], col[rows], label=label)


def step_checked(env, act, obs, rew, box, v, agents=None, label=""):
    """One env step with actions ``act`` (host), checked teacher-forced."""
    pre = gpu_state(env)
    env.step(dev(act), obs, rew)
    return check_post(env, pre, act, box, v, obs, rew, agents, label)


# --------------------------------------------------------------------------- reset

@pytest.mark.parametrize("name", ["flock256", "flock5k"])
def test_reset_view(name):
    cfg = workloads.WORKLOADS[name]
    st = workloads.make_state(name, seed=0)
    env, obs0 = make_env(st, cfg["box"], cfg["sectors"])
    torch.cuda.synchronize()
    nb, col = (host(t) for t in env.counts())
    o = band(st, cfg["box"], cfg["sectors"])
    zero_rew = np.zeros(cfg["n"])
    check_sense(o, host(obs0), 0.1 * nb - col, nb, col, label=f"{name} reset")
    assert (zero_rew == host(env.returns())).all()


# --------------------------------------------------------------------------- full runs

LANES = pytest.mark.parametrize("lanes", [0, 1], ids=["auto-lanes", "one-lane"])


@LANES
def test_flock256_all_steps(lanes):
    """256 agents, 64 x 64, 8 sectors, 100 steps: every step, every agent; the
    automatic sweep lanes (64 per agent for so few agents) and one lane."""
    cfg = workloads.WORKLOADS["flock256"]
    box, v, n = cfg["box"], cfg["sectors"], cfg["n"]
    st = workloads.make_state("flock256", seed=0)
    env, _ = make_env(st, box, v)
    if lanes:
        env.set_sweep_lanes(lanes)
    obs = torch.empty(n, v, device="cuda")
    rew = torch.empty(n, device="cuda")
    ret_oracle = np.zeros(n)
    for t in range(cfg["steps"]):
        act = workloads.random_actions(n, seed=0, step=t)
        step_checked(env, act, obs, rew, box, v, label=f"flock256 step {t}")
        ret_oracle += band(gpu_state(env), box, v).reward
    ret = host(env.returns())
    np.testing.assert_allclose(ret, ret_oracle, rtol=1e-5, atol=1e-5)


def _run_sampled(name, check_at, n_sample, seed=0):
    cfg = workloads.WORKLOADS[name]
    box, v, n = cfg["box"], cfg["sectors"], cfg["n"]
    st = workloads.make_state(name, seed=seed)
    env, _ = make_env(st, box, v)
    obs = torch.empty(n, v, device="cuda")
    rew = torch.empty(n, device="cuda")
    g = np.random.default_rng(seed + 99)
    last = max(check_at)
    stats = []
    for t in range(last + 1):
        act = workloads.random_actions(n, seed=seed, step=t)
        if t in check_at:
            agents = np.sort(g.choice(n, size=min(n_sample, n), replace=False)).astype(np.int32)
            stats.append(step_checked(env, act, obs, rew, box, v, agents=agents,
                                      label=f"{name} step {t}"))
        else:
            env.step(dev(act), obs, rew)
    return stats


def test_flock5k_sampled_steps():
    """5,000 agents, side 316, 16 sectors, 1,000 steps; all agents at six steps."""
    _run_sampled("flock5k", {0, 1, 2, 10, 100, 999}, 5000)


def test_blobs50k_sampled_steps():
    """50,000 agents in 64 blobs, side 1,000, 500 steps; 3,000 sampled agents at six steps."""
    _run_sampled("blobs50k", {0, 1, 2, 10, 100, 499}, 3000)


def test_uniform50k_sampled_steps():
    _run_sampled("uniform50k", {0, 1, 5}, 3000)


def test_flock5k_x200_graph_replay_sampled():
    """The 200 x 5,000-agent batch (side 316, 16 sectors) as it is timed: K steps
    captured in one graph, replayed twice with new actions written between the
    replays.  A twin batch of the same envs steps the same actions eagerly, each
    step checked teacher-forced against the oracle on 300 sampled agents in six
    envs (both ends of the batch, block-index seams); the replayed rewards of
    every step, the last view, every env's state and returns equal the twin's
    bitwise."""
    n, box, v, E, K = 5000, 316.0, 16, 200, 4
    sts = [workloads.uniform_state(n, box, seed=500 + k) for k in range(E)]
    envs = [make_env(st, box, v)[0] for st in sts]
    twins = [make_env(st, box, v)[0] for st in sts]
    batch, eager = flock.Batch(envs), flock.Batch(twins)
    G, off = batch.n, batch.offsets
    assert G == n * E
    obs = torch.empty(G, v, device="cuda")
    rew = torch.empty(K, G, device="cuda")
    act = torch.empty(K, G, 2, device="cuda")
    obs_e = torch.empty(G, v, device="cuda")
    rew_e = torch.empty(G, device="cuda")
    stream = torch.cuda.Stream()
    acts = [[workloads.random_actions(n, seed=5, step=t, env=k) for k in range(E)]
            for t in range(2 * K)]
    sample = [0, 1, 63, 64, 128, 199]
    g = np.random.default_rng(8)
    agents = {k: np.sort(g.choice(n, 300, replace=False)).astype(np.int32) for k in sample}
    for rep in range(2):
        act.copy_(dev(np.stack([np.concatenate(acts[rep * K + t]) for t in range(K)])))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            if rep == 0:
                batch.capture(K, act, obs, rew, stream)
            batch.run(K, act, obs, rew, stream)
        stream.synchronize()
        for t in range(K):
            pre = {k: gpu_state(twins[k]) for k in sample}
            eager.step(act[t], obs_e, rew_e)
            for k in sample:
                rows = slice(off[k], off[k + 1])
                check_post(twins[k], pre[k], acts[rep * K + t][k], box, v, obs_e[rows],
                           rew_e[rows], agents[k], label=f"env {k} replay {rep} step {t}")
            assert torch.equal(rew[t], rew_e), f"replay {rep} step {t}: rewards differ"
        assert torch.equal(obs, obs_e), f"replay {rep}: view differs"
    for k in range(E):
        assert all(torch.equal(a, b) for a, b in zip(envs[k].get_state(), twins[k].get_state()))
        assert torch.equal(envs[k].returns(), twins[k].returns())


# --------------------------------------------------------------------------- edge cases

def _one_step_case(st, box, v, reach=0, steps=3, seed=0, lanes=0):
    n = st[0].shape[0]
    env, obs0 = make_env(st, box, v, reach=reach)
    if lanes:
        env.set_sweep_lanes(lanes)
    torch.cuda.synchronize()
    if n > 0:
        nb, col = (host(t) for t in env.counts())
        check_sense(band(st, box, v), host(obs0), 0.1 * nb - col, nb, col, label="reset")
    obs = torch.empty(n, v, device="cuda")
    rew = torch.empty(n, device="cuda")
    for t in range(steps):
        act = workloads.random_actions(n, seed=seed, step=t)
        if n > 0:
            step_checked(env, act, obs, rew, box, v, label=f"step {t}")
        else:
            env.step(dev(act), obs, rew)
    torch.cuda.synchronize()
    return env


def test_empty_env():
    st = tuple(np.zeros(0, np.float32) for _ in range(4))
    _one_step_case(st, 64.0, 8)


@LANES
@pytest.mark.parametrize("n", [1, 2, 3])
def test_tiny_envs(n, lanes):
    st = workloads.uniform_state(n, 20.0, seed=n)
    _one_step_case(st, 20.0, 8, lanes=lanes)


@LANES
@pytest.mark.parametrize("box", [16.5, 20.0, 24.0, 24.5, 33.0])
def test_small_boxes_all_pairs_and_three_cells(box, lanes):
    n = int(box * box / 4)
    st = workloads.uniform_state(n, box, seed=3)
    env = _one_step_case(st, box, 16, lanes=lanes)
    ncell, _, reach, _, _ = env.geometry()
    assert (ncell == 1) == (box <= 24.0)
    assert ncell == 1 or ncell >= 3


@LANES
@pytest.mark.parametrize("v", [1, 3, 8, 16, 32, 33, 64, 128, 256])
def test_sector_counts(v, lanes):
    st = workloads.uniform_state(2000, 120.0, seed=v)
    _one_step_case(st, 120.0, v, steps=2, lanes=lanes)


@LANES
def test_reach_two_stencil(lanes):
    st = workloads.uniform_state(4000, 160.0, seed=4)
    env = _one_step_case(st, 160.0, 16, reach=2, lanes=lanes)
    assert env.geometry()[2] == 2


@LANES
def test_dense_cluster_and_coincident(lanes):
    """Skewed occupancy: most agents inside one cell, many exact duplicates."""
    g = np.random.default_rng(5)
    n, box = 3000, 200.0
    x = (100.0 + g.random(n) * 3.0).astype(np.float32)
    y = (50.0 + g.random(n) * 3.0).astype(np.float32)
    x[::7] = x[0]
    y[::7] = y[0]
    th = (g.random(n) * 6.28).astype(np.float32)
    s = np.zeros(n, np.float32)
    _one_step_case((x, y, th, s), box, 16, steps=2, lanes=lanes)


@LANES
def test_cell_boundaries_and_seams(lanes):
    """Agents exactly on column and row boundaries, at 0 and just below the box side."""
    box, v = 64.0, 16
    env0 = flock.Env(flock.Params(n_agents=10000, box=box, sectors=v))
    ncx, ncy, _, cw, ch = env0.geometry()
    top = np.nextafter(np.float32(box), np.float32(0))
    xs = np.array([k * cw for k in range(ncx)] + [0.0, top], np.float32)
    ys = np.array([k * ch for k in range(ncy)] + [0.0, top], np.float32)
    xx, yy = np.meshgrid(xs, ys, indexing="ij")
    x, y = xx.ravel().astype(np.float32), yy.ravel().astype(np.float32)
    n = x.shape[0]
    th = (np.arange(n) * 0.37 % 6.2).astype(np.float32)
    s = np.zeros(n, np.float32)
    _one_step_case((x, y, th, s), box, v, steps=2, lanes=lanes)


def test_single_large_env():
    """2^20 agents in one env (side 4,096): sampled agents after two steps."""
    n, box, v = 1 << 20, 4096.0, 16
    st = workloads.uniform_state(n, box, seed=8)
    env, _ = make_env(st, box, v)
    obs = torch.empty(n, v, device="cuda")
    rew = torch.empty(n, device="cuda")
    agents = np.sort(np.random.default_rng(1).choice(n, 2000, replace=False)).astype(np.int32)
    for t in range(2):
        act = workloads.random_actions(n, seed=8, step=t)
        step_checked(env, act, obs, rew, box, v, agents=agents, label=f"1M env step {t}")


def test_sparse_env_many_cells():
    """2^20 agents in side 16,384: 2,046 columns of 8,184 rows, 16.7M cells, so the
    cell scan runs with more tiles than its direct-offset limit; sampled agents."""
    n, box, v = 1 << 20, 16384.0, 16
    st = workloads.uniform_state(n, box, seed=9)
    env, _ = make_env(st, box, v)
    ncx, ncy, _, _, _ = env.geometry()
    assert ncx * ncy > 4096 * 2048
    obs = torch.empty(n, v, device="cuda")
    rew = torch.empty(n, device="cuda")
    agents = np.sort(np.random.default_rng(2).choice(n, 2000, replace=False)).astype(np.int32)
    for t in range(2):
        act = workloads.random_actions(n, seed=9, step=t)
        step_checked(env, act, obs, rew, box, v, agents=agents, label=f"16.7M-cell env step {t}")


# --------------------------------------------------------------------------- batched

def _uneven(n_envs, lo, hi, seed):
    ns, boxes = workloads.uneven_env_sizes(n_envs, lo, hi, seed=seed)
    states = [workloads.uniform_state(int(n), float(b), seed=seed, env=k)
              for k, (n, b) in enumerate(zip(ns, boxes))]
    return ns, boxes, states


def test_batched_equals_plain_bitwise():
    ns, boxes, states = _uneven(12, 20, 3000, seed=21)
    # add an empty env, a single-cell env and a reach-2 env
    extra = [(0, 64.0, 0), (150, 20.0, 0), (800, 100.0, 2)]
    envs_a, envs_b, boxes_all, states_all = [], [], [], []
    for k, (n, b) in enumerate(zip(ns, boxes)):
        boxes_all.append(float(b))
        states_all.append(states[k])
    for n, b, r in extra:
        boxes_all.append(b)
        states_all.append(workloads.uniform_state(n, b, seed=5))
    reaches = [0] * len(ns) + [e[2] for e in extra]
    for st, b, r in zip(states_all, boxes_all, reaches):
        envs_a.append(make_env(st, b, 16, reach=r)[0])
        envs_b.append(make_env(st, b, 16, reach=r)[0])
    batch = flock.Batch(envs_b)
    batch.set_sweep_lanes(1)   # one lane per agent against each env's automatic lane groups
    G = batch.n
    obs_b = torch.empty(G, 16, device="cuda")
    rew_b = torch.empty(G, device="cuda")
    off = batch.offsets
    for t in range(4):
        acts = [workloads.random_actions(st[0].shape[0], seed=1, step=t, env=k)
                for k, st in enumerate(states_all)]
        act_b = dev(np.concatenate(acts).reshape(G, 2))
        batch.step(act_b, obs_b, rew_b)
        for k, env in enumerate(envs_a):
            o, r = env.step(dev(acts[k]))
            assert torch.equal(o, obs_b[off[k]:off[k + 1]]), f"obs env {k} step {t}"
            assert torch.equal(r, rew_b[off[k]:off[k + 1]]), f"reward env {k} step {t}"
    for ea, eb in zip(envs_a, envs_b):
        assert torch.equal(ea.returns(), eb.returns())
        for u, w in zip(ea.get_state(), eb.get_state()):
            assert torch.equal(u, w)


@pytest.mark.parametrize("lanes", [4, 16, 64])
def test_sweep_lane_groups_bitwise_equal_to_one_lane(lanes):
    """Lane groups per agent give the same bits as one lane per agent.

    Envs: 50,000 agents in 64 blobs (hundreds of candidates per agent), a
    dense uniform env, a single-cell env, a reach-2 env, three tiny ones and
    an empty one, batched; the one-lane reference is each env stepped alone.
    """
    specs = [(50000, 1000.0, 0, "blobs"), (4000, 100.0, 0, "uniform"), (150, 20.0, 0, "uniform"),
             (800, 100.0, 2, "uniform"), (1, 64.0, 0, "uniform"), (2, 64.0, 0, "uniform"),
             (3, 30.0, 0, "uniform"), (0, 64.0, 0, "uniform")]
    states, ref, grp = [], [], []
    for k, (n, box, reach, init) in enumerate(specs):
        st = (workloads.blob_state(n, box, seed=k) if init == "blobs"
              else workloads.uniform_state(n, box, seed=k))
        states.append(st)
        e1 = make_env(st, box, 16, reach=reach)[0]
        e1.set_sweep_lanes(1)
        ref.append(e1)
        grp.append(make_env(st, box, 16, reach=reach)[0])
    batch = flock.Batch(grp)
    batch.set_sweep_lanes(lanes)
    G, off = batch.n, batch.offsets
    obs_b = torch.empty(G, 16, device="cuda")
    rew_b = torch.empty(G, device="cuda")
    agents = np.sort(np.random.default_rng(lanes).choice(50000, 1500, replace=False)).astype(np.int32)
    for t in range(3):
        acts = [workloads.random_actions(st[0].shape[0], seed=2, step=t, env=k)
                for k, st in enumerate(states)]
        pre = gpu_state(grp[0])
        batch.step(dev(np.concatenate(acts).reshape(G, 2)), obs_b, rew_b)
        for k, env in enumerate(ref):
            o, r = env.step(dev(acts[k]))
            assert torch.equal(o, obs_b[off[k]:off[k + 1]]), f"obs env {k} step {t}"
            assert torch.equal(r, rew_b[off[k]:off[k + 1]]), f"reward env {k} step {t}"
        if t == 2:   # and against the oracle on sampled agents of the clustered env
            check_post(grp[0], pre, acts[0], 1000.0, 16, obs_b[off[0]:off[1]],
                       rew_b[off[0]:off[1]], agents=agents, label=f"lanes {lanes}")
    for ea, eb in zip(ref, grp):
        assert torch.equal(ea.returns(), eb.returns())
        assert all(torch.equal(u, w) for u, w in zip(ea.counts(), eb.counts()))


@pytest.mark.parametrize("big", [0, 5000, 12000])
def test_per_env_fused_sort_batch_bitwise_and_oracle(big):
    """100+ small envs take the one-block-per-env sort; results equal each env stepped alone.

    Includes an empty env, single-cell envs, a reach-2 env, a tag-free mix of
    sizes 1 .. 3,000 and a view with more sectors; 6 steps, then the oracle on
    sampled agents of every tenth env.  The largest env sets the records per
    thread: up to 4,096 agents 4, with a 5,000-agent env 8 (records held in
    registers), with a 12,000-agent env 16 (records staged in memory).
    """
    ns, boxes, states = _uneven(100, 20, 3000, seed=33)
    extra = [(0, 64.0, 0), (1, 64.0, 0), (150, 20.0, 0), (800, 100.0, 2), (2, 30.0, 0)]
    if big:
        extra.append((big, float(np.sqrt(big * 16.0)), 0))
    sts = list(states) + [workloads.uniform_state(n, b, seed=6) for n, b, _ in extra]
    bxs = [float(b) for b in boxes] + [b for _, b, _ in extra]
    reaches = [0] * len(ns) + [r for _, _, r in extra]
    plain = [make_env(st, b, 16, reach=r)[0] for st, b, r in zip(sts, bxs, reaches)]
    fused = [make_env(st, b, 16, reach=r)[0] for st, b, r in zip(sts, bxs, reaches)]
    batch = flock.Batch(fused)
    G, off = batch.n, batch.offsets
    obs_b = torch.empty(G, 16, device="cuda")
    rew_b = torch.empty(G, device="cuda")
    g = np.random.default_rng(4)
    check = [k for k in sorted(set(range(0, len(sts), 10)) | {len(sts) - 1}) if sts[k][0].shape[0]]
    agents = {k: np.sort(g.choice(sts[k][0].shape[0], size=min(20, sts[k][0].shape[0]),
                                  replace=False)).astype(np.int32) for k in check}
    for t in range(6):
        acts = [workloads.random_actions(st[0].shape[0], seed=3, step=t, env=k)
                for k, st in enumerate(sts)]
        pre = {k: gpu_state(fused[k]) for k in check} if t == 5 else {}
        batch.step(dev(np.concatenate(acts).reshape(G, 2)), obs_b, rew_b)
        for k, env in enumerate(plain):
            o, r = env.step(dev(acts[k]))
            assert torch.equal(o, obs_b[off[k]:off[k + 1]]), f"obs env {k} step {t}"
            assert torch.equal(r, rew_b[off[k]:off[k + 1]]), f"reward env {k} step {t}"
        for k in pre:   # the last step against the oracle on sampled agents
            check_post(fused[k], pre[k], acts[k], bxs[k], 16, obs_b[off[k]:off[k + 1]],
                       rew_b[off[k]:off[k + 1]], agents=agents[k], label=f"fused env {k}")
    for ea, eb in zip(plain, fused):
        assert torch.equal(ea.returns(), eb.returns())
        assert all(torch.equal(u, w) for u, w in zip(ea.get_state(), eb.get_state()))


def test_batched_uneven_256_envs_against_oracle():
    """256 envs, N_e log-uniform in [100, 20,000] at density 1/16, 200 steps: 16
    sampled agents of every env checked teacher-forced at steps 0, 1, 2, 10 and
    199 (device-drawn actions in between)."""
    ns, boxes, states = _uneven(256, 100, 20000, seed=0)
    envs = [make_env(st, float(b), 16)[0] for st, b in zip(states, boxes)]
    batch = flock.Batch(envs)
    G = batch.n
    off = batch.offsets
    obs = torch.empty(G, 16, device="cuda")
    rew = torch.empty(G, device="cuda")
    g = np.random.default_rng(3)
    agents = [np.sort(g.choice(int(n), size=min(16, int(n)), replace=False)).astype(np.int32)
              for n in ns]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    scale = torch.tensor([0.2, 0.1], device="cuda")
    for t in range(200):
        if t not in (0, 1, 2, 10, 199):
            act = (torch.rand(G, 2, device="cuda", generator=gen) * 2.0 - 1.0) * scale
            batch.step(act, obs, rew)
            continue
        acts = [workloads.random_actions(int(n), seed=0, step=t, env=k) for k, n in enumerate(ns)]
        pre = [gpu_state(e) for e in envs]
        batch.step(dev(np.concatenate(acts)), obs, rew)
        for k in range(256):
            rows = slice(off[k], off[k + 1])
            check_post(envs[k], pre[k], acts[k], float(boxes[k]), 16, obs[rows], rew[rows],
                       agents=agents[k], label=f"env {k} step {t}")


@pytest.mark.parametrize("n_envs", [10, 80])   # 80: the one-block-per-env sort
def test_graph_replay_matches_eager(n_envs):
    ns, boxes, states = _uneven(n_envs, 50, 2000, seed=7)
    envs_g = [make_env(st, float(b), 16)[0] for st, b in zip(states, boxes)]
    envs_e = [make_env(st, float(b), 16)[0] for st, b in zip(states, boxes)]
    bg, be = flock.Batch(envs_g), flock.Batch(envs_e)
    G, K = bg.n, 5
    stream = torch.cuda.Stream()
    obs_g = torch.empty(G, 16, device="cuda")
    rew_g = torch.empty(K, G, device="cuda")
    obs_e = torch.empty(G, 16, device="cuda")
    rew_e = torch.empty(G, device="cuda")
    for rep in range(3):
        act = torch.stack([dev(np.concatenate([workloads.random_actions(int(n), seed=rep, step=t, env=k)
                                               for k, n in enumerate(ns)])) for t in range(K)])
        act = act.contiguous()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            bg.run(K, act, obs_g, rew_g, stream)
        stream.synchronize()
        for t in range(K):
            be.step(act[t].contiguous(), obs_e, rew_e)
            torch.cuda.synchronize()
            assert torch.equal(rew_e, rew_g[t]), f"rep {rep} step {t}"
        assert torch.equal(obs_e, obs_g)
        # eager work between replays
        _ = (obs_e * 2).sum().item()
    for a, b in zip(envs_g, envs_e):
        assert torch.equal(a.returns(), b.returns())


def test_returns_accumulate_fp64():
    st = workloads.uniform_state(500, 90.0, seed=2)
    env, _ = make_env(st, 90.0, 16)
    acc = np.zeros(500)
    for t in range(20):
        _, r = env.step(dev(workloads.random_actions(500, seed=2, step=t)))
        acc += host(r).astype(np.float64)
    np.testing.assert_array_equal(host(env.returns()), acc)


@pytest.mark.parametrize("n_envs", [10, 80])   # 80: the one-block-per-env sort
def test_timed_step_equals_step(n_envs):
    """env_step_batched_timed gives the results of env_step_batched and four phase
    times.  The scan and scatter phases are 0 under the one-kernel sorts: the
    one-block-per-env sort (80 envs) and the strip sort (10 envs, whose states
    env_reset has left in cell order)."""
    ns, boxes, states = _uneven(n_envs, 50, 2000, seed=9)
    envs_t = [make_env(st, float(b), 16)[0] for st, b in zip(states, boxes)]
    envs_s = [make_env(st, float(b), 16)[0] for st, b in zip(states, boxes)]
    bt, bs = flock.Batch(envs_t), flock.Batch(envs_s)
    G = bt.n
    obs_t, obs_s = torch.empty(G, 16, device="cuda"), torch.empty(G, 16, device="cuda")
    rew_t, rew_s = torch.empty(G, device="cuda"), torch.empty(G, device="cuda")
    for t in range(3):
        act = dev(np.concatenate([workloads.random_actions(int(n), seed=9, step=t, env=k)
                                  for k, n in enumerate(ns)]))
        ms = bt.step_timed(act, obs_t, rew_t)
        bs.step(act, obs_s, rew_s)
        torch.cuda.synchronize()
        assert torch.equal(obs_t, obs_s) and torch.equal(rew_t, rew_s), t
        assert len(ms) == 4 and all(m >= 0.0 for m in ms) and ms[0] > 0.0 and ms[3] > 0.0
        assert ms[1] == 0.0 and ms[2] == 0.0


@pytest.mark.parametrize("init", ["uniform", "blobs"])
def test_strip_sort_wait_fallback_bitwise(init):
    """The strip sort's fallback, forced from the host: with no look-back wait
    at all every strip but an env's first counts the agents before it itself.
    Over six steps the views, rewards, states and returns equal those of a
    twin batch that waits, bitwise, on envs of several strips each (uniform,
    and clustered so that strips overflow their LDS list)."""
    sizes = [(20000, 600.0), (6000, 300.0), (900, 120.0)]
    mk = workloads.blob_state if init == "blobs" else workloads.uniform_state
    states = [mk(n, b, seed=40 + k) for k, (n, b) in enumerate(sizes)]
    pair = []
    for _ in range(2):
        envs = [make_env(st, b, 16)[0] for st, (_, b) in zip(states, sizes)]
        pair.append((envs, flock.Batch(envs)))
    pair[1][1].set_strip_wait(0)
    G = pair[0][1].n
    obs = [torch.empty(G, 16, device="cuda") for _ in range(2)]
    rew = [torch.empty(G, device="cuda") for _ in range(2)]
    for t in range(6):
        act = dev(np.concatenate([workloads.random_actions(n, seed=41, step=t, env=k)
                                  for k, (n, _) in enumerate(sizes)]))
        for (_, b), o, r in zip(pair, obs, rew):
            b.step(act, o, r)
        torch.cuda.synchronize()
        assert torch.equal(obs[0], obs[1]) and torch.equal(rew[0], rew[1]), t
    for ea, eb in zip(pair[0][0], pair[1][0]):
        for x, y in zip(ea.get_state(), eb.get_state()):
            assert torch.equal(x, y)
        assert torch.equal(ea.returns(), eb.returns())


# --------------------------------------------------------------------------- move arithmetic

@LANES
def test_nan_inf_and_out_of_range_actions(lanes):
    """Actions outside their range, NaN and +-inf (read R13 of the oracle: clamp
    with fmin/fmax semantics, NaN to the lower bound) through env_step, three
    steps of 3,000 agents, each checked teacher-forced against the oracle's move
    and sense; the FP32 state stays finite and inside the box."""
    n, box, v = 3000, 200.0, 16
    st = workloads.uniform_state(n, box, seed=23)
    env, _ = make_env(st, box, v)
    if lanes:
        env.set_sweep_lanes(lanes)
    obs = torch.empty(n, v, device="cuda")
    rew = torch.empty(n, device="cuda")
    specials = np.array([np.nan, np.inf, -np.inf, 1e30, -1e30, 0.25, -0.25, 0.2, -0.2,
                         np.float32(0.2) * 2, -0.1, 0.1, 5.0, -5.0, 0.0, -0.0], np.float32)
    g = np.random.default_rng(29)
    for t in range(3):
        act = workloads.random_actions(n, seed=23, step=t)
        pick = g.random((n, 2)) < 0.5
        act = np.where(pick, specials[g.integers(0, specials.size, (n, 2))], act).astype(np.float32)
        act[:specials.size, 0] = specials
        act[specials.size:2 * specials.size, 1] = specials
        step_checked(env, act, obs, rew, box, v, label=f"special actions step {t}")
        post = gpu_state(env)
        assert all(np.isfinite(a).all() for a in post)
        assert ((post[3] >= 0.0) & (post[3] <= 2.0)).all()


def test_checkpoint_resume_with_returns():
    """Checkpoint after 7 steps (state and FP64 returns), resume in a fresh env
    (env_set_state, env_reset, env_set_returns) and run 5 more steps beside the
    original: views, rewards, state and returns stay bitwise equal (the step's
    results do not depend on the order agents are stored in)."""
    n, box, v = 4000, 250.0, 16
    st = workloads.uniform_state(n, box, seed=41)
    env, _ = make_env(st, box, v)
    for t in range(7):
        env.step(dev(workloads.random_actions(n, seed=41, step=t)))
    saved = env.get_state()
    saved_ret = env.returns()
    torch.cuda.synchronize()
    assert host(saved_ret).any()
    res = flock.Env(flock.Params(n_agents=n, box=box, sectors=v, flags=1))
    res.set_state(*saved)
    res.reset()
    assert not host(res.returns()).any()
    res.set_returns(saved_ret)
    for t in range(7, 12):
        act = dev(workloads.random_actions(n, seed=41, step=t))
        o1, r1 = env.step(act)
        o2, r2 = res.step(act)
        torch.cuda.synchronize()
        assert np.array_equal(host(o1).view(np.int32), host(o2).view(np.int32)), t
        assert np.array_equal(host(r1).view(np.int32), host(r2).view(np.int32)), t
    for a, b in zip(gpu_state(env), gpu_state(res)):
        assert np.array_equal(a.view(np.int32), b.view(np.int32))
    assert np.array_equal(host(env.returns()).view(np.int64), host(res.returns()).view(np.int64))


def test_move_cos_sin_within_one_ulp():
    """The move's FP32 cos/sin against the correctly rounded values the oracle uses.

    An agent at x = 0 with speed 1 and no action lands at x' = cos h whenever
    cos h >= 0 (x + 1 * cos h is then exact), so its new x exposes the
    kernel's cosine; likewise y = 0 exposes the sine.  131,072 headings spread
    over the first quadrant (the others use the same polynomials with swapped
    roles and signs) plus its edges, in two envs: x = 0 with the agents spread
    over 128 rows 0.5 apart (vision 0.4, so a row's agents see only each
    other), and y = 0 with them spread over columns.  Every exposed value
    within 1 ulp of the oracle's.  The share that is correctly rounded is
    checked against what an exact FP32 emulation of the same operations
    gives for these headings (84.4 % for cos, 94.0 % for sin: the final
    rounding of the reduced argument alone costs up to 0.35 ulp near pi/4),
    so a changed polynomial or reduction shows up as a changed share.
    """
    g = np.random.default_rng(17)
    h = np.concatenate([g.random(131_068) * (np.pi / 2), [0.0, np.pi / 4, np.pi / 2,
                        float(np.nextafter(np.float32(np.pi / 2), np.float32(0)))]])
    h = h.astype(np.float32)
    h = h[(np.cos(h.astype(np.float64)) >= 0) & (np.sin(h.astype(np.float64)) >= 0)]
    n = h.shape[0]
    lane = (0.5 * (np.arange(n) % 128)).astype(np.float32)
    zero = np.zeros(n, np.float32)
    act = np.zeros((n, 2), np.float32)
    for k, name, st in ((0, "cos", (zero, lane, h, np.ones(n, np.float32))),
                        (1, "sin", (lane, zero.copy(), h, np.ones(n, np.float32)))):
        env = flock.Env(flock.Params(n_agents=n, box=128.0, radius=0.4, collide=0.4, sectors=8))
        env.set_state(*[dev(a) for a in st])
        env.reset()
        env.step(dev(act))
        got = gpu_state(env)[k].view(np.int32).astype(np.int64)
        want = oracle.oracle_move(st, act, 128.0)[k].view(np.int32).astype(np.int64)
        ulp = np.abs(got - want)
        assert ulp.max() <= 1, f"{name}: {ulp.max()} ulp at heading {h[np.argmax(ulp)]!r}"
        share = float((ulp == 0).mean())
        assert share > {"cos": 0.83, "sin": 0.93}[name], f"{name}: only {share:.4f} correctly rounded"
