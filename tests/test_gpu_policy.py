"""GPU policy network (BF16 MFMA, FP32 accumulate) against the FP64 oracle.

Error bound.  With u = 2^-9 (half an ulp of BF16, relative) every input,
weight and hidden activation carries a relative rounding of at most u, and
FP32 accumulation adds at most K * 2^-24 relative.  Propagating first-order
absolute errors through z = W^T h + b (tanh is 1-Lipschitz) gives, per agent
and unit, with dh the error of the layer input (its own BF16 rounding
included),
    |dz| <= |W|^T dh + (u + K 2^-24) |W|^T |h| + 1e-6   (tanh evaluation)
and the action error is at most scale * |dz_out|.  The test computes this
bound in FP64 for every agent and requires the GPU error to stay under it.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu
flock = pytest.importorskip("paper_2207_03945_amd")

U_BF16 = 2.0 ** -9


def error_bound(obs, ws, bs, scale=(0.2, 0.1)):
    h = np.asarray(obs, np.float64)
    dh = U_BF16 * np.abs(h)                  # input rounding
    for layer, (w, b) in enumerate(zip(ws, bs)):
        w = np.asarray(w, np.float64)
        aw = np.abs(w)
        k = w.shape[0]
        dz = dh @ aw + (U_BF16 + k * 2.0 ** -24) * (np.abs(h) @ aw) + 1e-6
        h = np.tanh(h @ w + b)
        dh = dz + (U_BF16 * np.abs(h) if layer < len(ws) - 1 else 0.0)  # hidden layers re-rounded to BF16
    return dh * np.asarray(scale)


def make_policy(in_dim, seed=0):
    ws, bs = workloads.xavier_weights([in_dim, 64, 64, 2], seed=seed)
    bs = [b + np.float32(0.05) * (k + 1) for k, b in enumerate(bs)]  # non-zero biases
    return flock.Policy(ws, bs), ws, bs


@pytest.mark.parametrize("in_dim,n", [(16, 4096), (16, 1), (16, 77), (8, 1000), (20, 333), (32, 64),
                                      (33, 100), (48, 200), (128, 500), (129, 3000), (257, 64)])
def test_policy_matches_fp64_within_bound(in_dim, n):
    pol, ws, bs = make_policy(in_dim)
    g = np.random.default_rng(in_dim * 1000 + n)
    obs = g.random((n, in_dim)).astype(np.float32)
    obs[g.random((n, in_dim)) < 0.3] = 0.0          # empty sectors read 0
    act = pol.forward(torch.from_numpy(obs).cuda())
    torch.cuda.synchronize()
    got = act.cpu().numpy().astype(np.float64)
    ref = oracle.policy_forward(obs, ws, bs)
    bound = error_bound(obs, ws, bs)
    err = np.abs(got - ref)
    assert (err <= bound).all(), f"max err {err.max():.3e}, bound at worst {bound[err > bound][:3]}"
    print(f"in={in_dim} n={n}: max |act err| {err.max():.2e} (turn) / mean bound {bound.mean():.2e}")


@pytest.mark.parametrize("in_dim", [16, 129])
def test_policy_many_tiles_per_wave(in_dim):
    """More rows than one pass of the grid covers (4,096 blocks x 4 waves x 16
    rows, then a ragged tail): each wave loops over several tiles, reusing its
    LDS tiles.  Sampled rows equal the same rows evaluated on their own and stay
    within the FP64 bound."""
    pol, ws, bs = make_policy(in_dim)
    n = 300_000 + 37
    g = np.random.default_rng(11 + in_dim)
    obs_h = g.random((n, in_dim)).astype(np.float32)
    obs = torch.from_numpy(obs_h).cuda()
    act = pol.forward(obs)
    rows = np.sort(np.concatenate([g.choice(n - 64, 4000, replace=False), np.arange(n - 64, n)]))
    idx = torch.from_numpy(rows).cuda()
    sub = pol.forward(obs[idx].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(act[idx], sub)
    got = act.cpu().numpy()[rows].astype(np.float64)
    ref = oracle.policy_forward(obs_h[rows], ws, bs)
    bound = error_bound(obs_h[rows], ws, bs)
    err = np.abs(got - ref)
    assert (err <= bound).all(), f"max err {err.max():.3e}"


def test_policy_row_independent_bitwise():
    """An agent's action does not depend on its tile or the batch size."""
    pol, _, _ = make_policy(16)
    g = np.random.default_rng(3)
    obs = torch.from_numpy(g.random((1000, 16)).astype(np.float32)).cuda()
    a_full = pol.forward(obs)
    perm = torch.from_numpy(g.permutation(1000)).cuda()
    a_perm = pol.forward(obs[perm].contiguous())
    assert torch.equal(a_perm, a_full[perm])
    a_part = pol.forward(obs[37:70].contiguous())
    assert torch.equal(a_part, a_full[37:70])


def test_policy_empty_input():
    pol, _, _ = make_policy(16)
    act = pol.forward(torch.empty(0, 16, device="cuda"))
    torch.cuda.synchronize()
    assert act.shape == (0, 2)


def test_step_policy_equals_forward_then_step():
    ns, boxes = [300, 1200, 64], [70.0, 140.0, 33.0]
    pol, _, _ = make_policy(16)
    envs_a, envs_b = [], []
    for k, (n, b) in enumerate(zip(ns, boxes)):
        st = workloads.uniform_state(n, b, seed=k)
        for lst in (envs_a, envs_b):
            e = flock.Env(flock.Params(n_agents=n, box=b, sectors=16))
            e.set_state(*[torch.from_numpy(a).cuda() for a in st])
            lst.append(e)
    obs_a = torch.cat([e.reset() for e in envs_a]).contiguous()
    obs_b = torch.cat([e.reset() for e in envs_b]).contiguous()
    ba, bb = flock.Batch(envs_a), flock.Batch(envs_b)
    G = ba.n
    act_a = torch.empty(G, 2, device="cuda")
    rew_a = torch.empty(G, device="cuda")
    rew_b = torch.empty(G, device="cuda")
    for t in range(5):
        ba.step_policy(pol, act_a, obs_a, rew_a)
        act_b = pol.forward(obs_b)
        bb.step(act_b, obs_b, rew_b)
        torch.cuda.synchronize()
        assert torch.equal(act_a, act_b), t
        assert torch.equal(obs_a, obs_b), t
        assert torch.equal(rew_a, rew_b), t


@pytest.mark.parametrize("in_dim", [16, 129, 20])
def test_policy_staged_and_direct_loads_agree_bitwise(in_dim):
    """Rows staged through LDS (16-byte aligned obs) and rows loaded per lane
    (obs starting 4 bytes in) give the same actions."""
    pol, _, _ = make_policy(in_dim)
    n = 1000
    g = np.random.default_rng(in_dim)
    obs = torch.from_numpy(g.random((n, in_dim)).astype(np.float32)).cuda()
    big = torch.empty(n * in_dim + 1, device="cuda")
    shifted = big[1:].view(n, in_dim)
    shifted.copy_(obs)
    assert shifted.data_ptr() % 16 != 0
    a = pol.forward(obs)
    b = pol.forward(shifted)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("kind,lanes", [("v16", 0), ("v16", 1), ("v16", 4), ("v16", 64),
                                        ("v8", 16), ("v8", 1), ("paper129", 16), ("paper129", 1),
                                        ("paper129", 4)])
def test_fused_policy_step_equals_forward_then_step(kind, lanes):
    """env_step_policy with policy fusion on (the next step's actions come from
    the views still on chip when the sweep has one or four lanes per agent; a
    separate launch with 16 or 64): over six steps its actions, views and
    rewards equal pol_forward + env_step_batched bitwise, for each sweep lane
    count and view kind; the cached next actions are recomputed when the obs
    pointer changes and when an env's state is set anew."""
    if kind == "paper129":
        ps = [flock.Params(n_agents=n, box=100.0, radius=10.0, sectors=128,
                           fov=math.radians(250.0), flags=flock.ENV_FLAG_SPEED_OBS)
              for n in (900, 70)]
        in_dim = 129
    else:
        v = 16 if kind == "v16" else 8
        ps = [flock.Params(n_agents=n, box=b, sectors=v) for n, b in ((2500, 200.0), (333, 75.0))]
        in_dim = v
    pol, _, _ = make_policy(in_dim)
    states = [workloads.uniform_state(p.n_agents, p.box, seed=k + 3) for k, p in enumerate(ps)]
    pair = []
    for _ in range(2):
        envs = []
        for p, st in zip(ps, states):
            e = flock.Env(p)
            e.set_state(*[torch.from_numpy(a).cuda() for a in st])
            envs.append(e)
        obs = torch.cat([e.reset() for e in envs]).contiguous()
        b = flock.Batch(envs)
        if lanes:
            b.set_sweep_lanes(lanes)
        pair.append((envs, b, obs))
    pair[0][1].set_policy_fusion(True)
    (envs_a, ba, obs_a), (envs_b, bb, obs_b) = pair
    G = ba.n
    act_a = torch.empty(G, 2, device="cuda")
    rew_a, rew_b = torch.empty(G, device="cuda"), torch.empty(G, device="cuda")
    for t in range(6):
        if t == 3:      # a new obs buffer: the policy is evaluated again
            obs_a = obs_a.clone()
        if t == 4:      # a state set anew on both sides
            st = workloads.uniform_state(ps[1].n_agents, ps[1].box, seed=99)
            for envs in (envs_a, envs_b):
                envs[1].set_state(*[torch.from_numpy(a).cuda() for a in st])
            off = ba.offsets
            for envs, o in ((envs_a, obs_a), (envs_b, obs_b)):
                o[off[1]:off[2]] = envs[1].reset()
        ba.step_policy(pol, act_a, obs_a, rew_a)
        act_b = pol.forward(obs_b)
        bb.step(act_b, obs_b, rew_b)
        torch.cuda.synchronize()
        assert torch.equal(act_a, act_b), t
        assert torch.equal(obs_a, obs_b), t
        assert torch.equal(rew_a, rew_b), t
