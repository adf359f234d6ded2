"""GPU experience collection: sampling, critic, rollout buffers, advantages.

* critic and sampled actions against the FP64 oracle (``oracle.rl``), within
  the first-order BF16 error bound used for the actor;
* env_rollout against the same steps taken one call at a time (bitwise), and
  teacher-forced against the oracle at every step (the oracle moves the
  GPU's pre-step state with the GPU's own actions: heading and speed bitwise,
  positions within the move tolerance; the view of the GPU's post-move state
  within the bands; the actions within the bound);
* rl_gae bitwise against the oracle: both evaluate the same FP64 operations
  in the same order on the same FP32 inputs and round once.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import rl
from parity import EPS_D, EPS_PHI, check_move, check_sense

pytestmark = pytest.mark.gpu
flock = pytest.importorskip("paper_2207_03945_amd")

U_BF16 = 2.0 ** -9
LOG_STD = (np.float32(-1.6), np.float32(-2.3))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def net_error_bound(obs, ws, bs, linear_out):
    """First-order bound on the BF16/FP32 network's output error (see test_gpu_policy)."""
    h = np.asarray(obs, np.float64)
    dh = U_BF16 * np.abs(h)
    n_layers = len(ws)
    for layer, (w, b) in enumerate(zip(ws, bs)):
        w = np.asarray(w, np.float64)
        aw = np.abs(w)
        k = w.shape[0]
        dz = dh @ aw + (U_BF16 + k * 2.0 ** -24) * (np.abs(h) @ aw) + 1e-6
        z = h @ w + b
        last = layer == n_layers - 1
        h = z if (last and linear_out) else np.tanh(z)
        dh = dz + (U_BF16 * np.abs(h) if layer < n_layers - 1 else 0.0)
    return dh


def actor(in_dim, seed=0):
    ws, bs = workloads.xavier_weights([in_dim, 64, 64, 2], seed=seed)
    bs = [b + np.float32(0.03) * (k + 1) for k, b in enumerate(bs)]
    return flock.Policy(ws, bs), ws, bs


def critic(in_dim, seed=1):
    ws, bs = workloads.xavier_weights([in_dim, 64, 64, 1], seed=seed)
    bs = [b + np.float32(0.02) * (k + 1) for k, b in enumerate(bs)]
    return flock.Critic(ws, bs), ws, bs


@pytest.mark.parametrize("in_dim,n", [(16, 4096), (129, 1000), (129, 33), (7, 1)])
def test_critic_matches_fp64_within_bound(in_dim, n):
    cr, ws, bs = critic(in_dim)
    g = np.random.default_rng(n)
    obs = g.random((n, in_dim)).astype(np.float32)
    obs[g.random((n, in_dim)) < 0.3] = 0.0
    got = host(cr.value(dev(obs))).astype(np.float64)
    ref = rl.value_forward(obs, ws, bs)
    bound = net_error_bound(obs, ws, bs, linear_out=True)[:, 0]
    err = np.abs(got - ref)
    assert (err <= bound).all(), f"max err {err.max():.3e}"


@pytest.mark.parametrize("in_dim,n", [(16, 2048), (129, 777)])
def test_sampled_actions_and_log_density(in_dim, n):
    pol, ws, bs = actor(in_dim)
    g = np.random.default_rng(in_dim)
    obs = g.random((n, in_dim)).astype(np.float32)
    eps = workloads.policy_noise(1, n, seed=3)[0]
    act, logp = pol.sample(dev(obs), dev(eps), LOG_STD)
    act, logp = host(act).astype(np.float64), host(logp).astype(np.float64)
    mean = oracle.policy_forward(obs, ws, bs)
    ref_a, ref_lp = rl.gaussian_sample(mean, np.array(LOG_STD, np.float64), eps)
    bound = net_error_bound(obs, ws, bs, linear_out=False) * np.array([0.2, 0.1])
    # plus the FP32 roundings of sigma, sigma * eps and the sum
    bound = bound + 4 * 2.0 ** -24 * (np.abs(ref_a) + np.abs(ref_a - mean))
    assert (np.abs(act - ref_a) <= bound).all()
    np.testing.assert_allclose(logp, ref_lp, rtol=4e-7, atol=4e-7)


def _paper_envs(sizes, seed, fov_deg=250.0):
    cfg = workloads.WORKLOADS["paper_flock1k"]
    ps = [flock.Params(n_agents=n, box=cfg["box"], radius=cfg["radius"], sectors=cfg["sectors"],
                       fov=math.radians(fov_deg),
                       flags=flock.ENV_FLAG_COUNTS | flock.ENV_FLAG_SPEED_OBS) for n in sizes]
    states = [workloads.uniform_state(n, cfg["box"], seed=seed, env=k) for k, n in enumerate(sizes)]
    return ps, states


def _make(ps, states):
    envs = []
    for p, st in zip(ps, states):
        e = flock.Env(p)
        e.set_state(*[dev(a) for a in st])
        envs.append(e)
    return envs


@pytest.mark.parametrize("fuse,lanes", [(False, 0), (True, 1), (True, 4)],
                         ids=["separate", "fused-1-lane", "fused-4-lanes"])
def test_rollout_equals_stepwise_and_oracle_teacher_forced(fuse, lanes):
    """The rollout against the same steps taken one call at a time, bitwise,
    with the policy launched separately or run inside the view sweep (one lane
    per agent: 129 inputs in five chunks; four lanes: the block-barrier path)."""
    sizes = [700, 1000, 37]
    ps, states = _paper_envs(sizes, seed=4)
    T = 8
    d = ps[0].obs_dim
    pol, ws, bs = actor(d, seed=2)
    envs_r, envs_s = _make(ps, states), _make(ps, states)
    for e_r, e_s in zip(envs_r, envs_s):
        e_r.reset()
        e_s.reset()
    br, bs_ = flock.Batch(envs_r), flock.Batch(envs_s)
    br.set_policy_fusion(fuse)
    if lanes:
        br.set_sweep_lanes(lanes)
    G, off = br.n, br.offsets
    eps = dev(workloads.policy_noise(T, G, seed=5))
    obs_buf = torch.empty(T + 1, G, d, device="cuda")
    act_buf = torch.empty(T, G, 2, device="cuda")
    logp_buf = torch.empty(T, G, device="cuda")
    rew_buf = torch.empty(T, G, device="cuda")
    # block 0: the batch-order view of the reset state
    obs0 = torch.cat([e.reset() for e in _make(ps, states)])
    obs_buf[0].copy_(obs0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        br.rollout(pol, T, obs_buf, act_buf, rew_buf, logp=logp_buf, eps=eps, log_std=LOG_STD,
                   stream=stream)
    stream.synchronize()

    # the same steps one call at a time, checked against the oracle as they go
    obs = obs0.clone()
    rew = torch.empty(G, device="cuda")
    g = np.random.default_rng(9)
    for t in range(T):
        act, logp = pol.sample(obs, eps[t].contiguous(), LOG_STD)
        mean = oracle.policy_forward(host(obs), ws, bs)
        ref_a, _ = rl.gaussian_sample(mean, np.array(LOG_STD, np.float64), host(eps[t]))
        bound = net_error_bound(host(obs), ws, bs, False) * np.array([0.2, 0.1]) + 1e-6
        assert (np.abs(host(act) - ref_a) <= bound).all(), f"action step {t}"
        pre = [tuple(host(a) for a in env.get_state()) for env in envs_s]
        bs_.step(act, obs, rew)
        torch.cuda.synchronize()
        assert torch.equal(act, act_buf[t]) and torch.equal(logp, logp_buf[t]), f"step {t}"
        assert torch.equal(obs, obs_buf[t + 1]) and torch.equal(rew, rew_buf[t]), f"step {t}"
        act_h, obs_h, rew_h = host(act), host(obs), host(rew)
        for k, env in enumerate(envs_s):
            lo, hi = off[k], off[k + 1]
            got = tuple(host(a) for a in env.get_state())
            check_move(got, oracle.oracle_move(pre[k], act_h[lo:hi], ps[k].box), ps[k].box,
                       f"state env {k} step {t}")
            agents = np.sort(g.choice(hi - lo, size=min(40, hi - lo), replace=False)).astype(np.int32)
            o = oracle.oracle_sense(got[0], got[1], got[2], ps[k].box, radius=ps[k].radius,
                                    sectors=ps[k].sectors, fov=ps[k].fov, agents=agents,
                                    eps_d=EPS_D, eps_phi=EPS_PHI)
            nb, col = (host(x) for x in env.counts())
            rows = lo + agents
            check_sense(o, obs_h[rows, :-1], rew_h[rows], nb[agents], col[agents],
                        radius=ps[k].radius, label=f"env {k} step {t}")
            assert np.array_equal(obs_h[rows, -1], got[3][agents])
    for e_r, e_s in zip(envs_r, envs_s):
        assert torch.equal(e_r.returns(), e_s.returns())
        assert all(torch.equal(u, w) for u, w in zip(e_r.get_state(), e_s.get_state()))


def test_rollout_graph_replay_and_mean_actions():
    """A second rollout on the same buffers replays the captured graph with new contents."""
    ps, states = _paper_envs([500, 900], seed=6)
    d = ps[0].obs_dim
    pol, _, _ = actor(d, seed=4)
    envs_r, envs_s = _make(ps, states), _make(ps, states)
    obs_r = torch.cat([e.reset() for e in envs_r])
    obs_s = torch.cat([e.reset() for e in envs_s])
    br, bs_ = flock.Batch(envs_r), flock.Batch(envs_s)
    G, T = br.n, 5
    obs_buf = torch.empty(T + 1, G, d, device="cuda")
    act_buf = torch.empty(T, G, 2, device="cuda")
    rew_buf = torch.empty(T, G, device="cuda")
    eps = torch.empty(T, G, 2, device="cuda")
    stream = torch.cuda.Stream()
    act_s = torch.empty(G, 2, device="cuda")
    rew_s = torch.empty(G, device="cuda")
    for seg in range(3):
        sample = seg != 1           # segment 1 takes the mean action
        eps.copy_(dev(workloads.policy_noise(T, G, seed=20 + seg)))
        obs_buf[0].copy_(obs_r)
        with torch.cuda.stream(stream):
            br.rollout(pol, T, obs_buf, act_buf, rew_buf, eps=eps if sample else None,
                       log_std=LOG_STD if sample else None, stream=stream)
        stream.synchronize()
        obs_r = obs_buf[T].clone()
        for t in range(T):
            if sample:
                act_s, _ = pol.sample(obs_s, eps[t].contiguous(), LOG_STD)
                bs_.step(act_s, obs_s, rew_s)
            else:
                bs_.step_policy(pol, act_s, obs_s, rew_s)
            torch.cuda.synchronize()
            assert torch.equal(act_s, act_buf[t]) and torch.equal(rew_s, rew_buf[t]), (seg, t)
            assert torch.equal(obs_s, obs_buf[t + 1]), (seg, t)


@pytest.mark.parametrize("T,n", [(128, 10007), (5, 300), (8, 64), (13, 1), (1, 257)])
def test_gae_bitwise_against_oracle(T, n):
    g = np.random.default_rng(T * 7 + n)
    rew = (g.random((T, n)) - 0.3).astype(np.float32)
    val = g.normal(size=(T + 1, n)).astype(np.float32)
    gamma, lam = np.float32(0.99), np.float32(0.95)
    adv, ret = flock.gae(dev(rew), dev(val), gamma, lam)
    ref_adv, ref_ret = rl.gae(rew, val, float(gamma), float(lam))
    assert np.array_equal(host(adv), ref_adv.astype(np.float32))
    assert np.array_equal(host(ret), ref_ret.astype(np.float32))


def test_collect_values_advantages_pipeline():
    """rollout -> critic over the whole obs buffer -> advantages, against the oracle."""
    ps, states = _paper_envs([1000, 400], seed=8)
    d = ps[0].obs_dim
    pol, _, _ = actor(d, seed=6)
    cr, cws, cbs = critic(d, seed=7)
    envs = _make(ps, states)
    obs0 = torch.cat([e.reset() for e in envs])
    b = flock.Batch(envs)
    G, T = b.n, 16
    obs_buf = torch.empty(T + 1, G, d, device="cuda")
    act_buf = torch.empty(T, G, 2, device="cuda")
    logp_buf = torch.empty(T, G, device="cuda")
    rew_buf = torch.empty(T, G, device="cuda")
    obs_buf[0].copy_(obs0)
    eps = dev(workloads.policy_noise(T, G, seed=11))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.rollout(pol, T, obs_buf, act_buf, rew_buf, logp=logp_buf, eps=eps, log_std=LOG_STD,
                  stream=stream)
        val = cr.value(obs_buf, stream=stream)
        adv, ret = flock.gae(rew_buf, val, 0.99, 0.95, stream=stream)
    stream.synchronize()
    obs_h = host(obs_buf).reshape(-1, d)
    v_ref = rl.value_forward(obs_h, cws, cbs).reshape(T + 1, G)
    bound = net_error_bound(obs_h, cws, cbs, True)[:, 0].reshape(T + 1, G)
    assert (np.abs(host(val) - v_ref) <= bound).all()
    a_ref, r_ref = rl.gae(host(rew_buf), host(val), float(np.float32(0.99)), float(np.float32(0.95)))
    assert np.array_equal(host(adv), a_ref.astype(np.float32))
    assert np.array_equal(host(ret), r_ref.astype(np.float32))
    # log densities of the samples
    lp_ref = rl.gaussian_sample(np.zeros((T * G, 2)), np.array(LOG_STD, np.float64),
                                host(eps).reshape(-1, 2))[1].reshape(T, G)
    np.testing.assert_allclose(host(logp_buf), lp_ref, rtol=4e-7, atol=4e-7)
