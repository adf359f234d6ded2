"""Serving loop: continuous batching with footprint admission (GPU).

The same request must give bitwise the same FP64 returns whether it runs
alone or overlapped with others (deterministic bursts force the overlap),
and the same as the plain env + policy closed loop; that closed loop is
checked against the oracle at every step, teacher-forced (actions within the
first-order BF16 bound of the FP64 network, move within the move tolerance,
view and reward within the bands), so the served returns are tied to the
oracle through it.
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


def policy():
    ws, bs = workloads.xavier_weights([16, 64, 64, 2], seed=0)
    return flock.Policy(ws, bs)


def request(n, seed):
    box = float(np.float32(4.0 * math.sqrt(n)))
    return flock.Params(n_agents=n, box=box, sectors=16), workloads.uniform_state(n, box, seed=seed)


def drain(srv, ids, max_ticks=100000):
    running_seen = []
    for _ in range(max_ticks):
        states = [srv.poll(i)[0] for i in ids]
        if all(s == srv.FINISHED for s in states):
            break
        n_run, _ = srv.tick()
        running_seen.append(n_run)
    return {i: srv.result(i) for i in ids}, running_seen


def test_alone_equals_in_the_mix_bitwise():
    pol = policy()
    target = request(3000, seed=11)
    alone = flock.Server(pol, 512 << 20, max_slots=8)
    rid, admitted = alone.submit(target[0], target[1], steps=25)
    assert admitted
    ret_alone, _ = drain(alone, [rid])

    mix = flock.Server(pol, 512 << 20, max_slots=8)
    others = [request(n, seed=20 + k) for k, n in enumerate([800, 5000, 1500, 12000])]
    ids = [mix.submit(p, st, steps=30)[0] for p, st in others[:2]]
    for _ in range(4):
        mix.tick()
    tid = mix.submit(target[0], target[1], steps=25)[0]      # joins a running batch
    mix.tick()
    ids += [mix.submit(p, st, steps=10)[0] for p, st in others[2:]]  # burst mid-episode
    res, seen = drain(mix, ids + [tid])
    assert max(seen) >= 4, "requests did not overlap"
    assert np.array_equal(res[tid], ret_alone[rid])


def test_served_equals_plain_closed_loop():
    pol = policy()
    p, st = request(2000, seed=5)
    srv = flock.Server(pol, 256 << 20, max_slots=4)
    rid, _ = srv.submit(p, st, steps=12)
    res, _ = drain(srv, [rid])
    env = flock.Env(p)
    env.set_state(*[torch.from_numpy(a).cuda() for a in st])
    obs = env.reset()
    for _ in range(12):
        act = pol.forward(obs)
        obs, _ = env.step(act)
    torch.cuda.synchronize()
    assert np.array_equal(res[rid], env.returns().cpu().numpy())


def test_admission_by_footprint_queues_and_completes():
    pol = policy()
    reqs = [request(n, seed=40 + k) for k, n in enumerate([6000, 6000, 6000, 6000, 700])]
    per = max(flock.request_bytes(p) for p, _ in reqs)
    srv = flock.Server(pol, int(2.3 * per), max_slots=16)     # room for about two at once
    ids, admitted = [], []
    for p, st in reqs:
        i, a = srv.submit(p, st, steps=6)
        ids.append(i)
        admitted.append(a)
    assert admitted[0] and not all(admitted)
    res, seen = drain(srv, ids)
    assert max(seen) <= 3 and len(res) == len(reqs)
    # the queued requests' results equal a run with ample memory
    big = flock.Server(pol, 1 << 30, max_slots=16)
    ids2 = [big.submit(p, st, steps=6)[0] for p, st in reqs]
    res2, _ = drain(big, ids2)
    for a, b in zip(ids, ids2):
        assert np.array_equal(res[a], res2[b])


def test_slot_limit_and_errors():
    pol = policy()
    srv = flock.Server(pol, 256 << 20, max_slots=2)
    ids = [srv.submit(*request(500, seed=k), steps=3)[0] for k in range(5)]
    res, seen = drain(srv, ids)
    assert max(seen) <= 2 and len(res) == 5
    with pytest.raises(flock.FlockError):
        srv.submit(flock.Params(n_agents=100, box=40.0, sectors=8),
                   workloads.uniform_state(100, 40.0), steps=3)
    tiny = flock.Server(pol, 1 << 16, max_slots=2)
    with pytest.raises(flock.FlockError) as ei:
        tiny.submit(*request(20000, seed=1), steps=3)
    assert ei.value.code == flock.flockenv.ENV_ENOMEM


def test_paper_flock_requests_served_with_speed_view():
    """129-input policy serving limited-view, speed-in-view requests; layouts are checked."""
    ws, bs = workloads.xavier_weights([129, 64, 64, 2], seed=3)
    pol = flock.Policy(ws, bs)
    fov = math.radians(250.0)
    p = flock.Params(n_agents=800, box=100.0, radius=10.0, sectors=128, fov=fov,
                     flags=flock.ENV_FLAG_SPEED_OBS)
    st = workloads.uniform_state(800, 100.0, seed=8)
    srv = flock.Server(pol, 256 << 20, max_slots=4)
    rid, _ = srv.submit(p, st, steps=6)
    # same row length, other layout (129 sectors, no speed): rejected
    with pytest.raises(flock.FlockError):
        srv.submit(flock.Params(n_agents=100, box=100.0, radius=10.0, sectors=129),
                   workloads.uniform_state(100, 100.0, seed=9), steps=3)
    res, _ = drain(srv, [rid])
    env = flock.Env(p)
    env.set_state(*[torch.from_numpy(a).cuda() for a in st])
    obs = env.reset()
    for _ in range(6):
        obs, _ = env.step(pol.forward(obs))
    torch.cuda.synchronize()
    assert np.array_equal(res[rid], env.returns().cpu().numpy())


U_BF16 = 2.0 ** -9


def _act_bound(obs, ws, bs):
    """First-order bound of the BF16/FP32 actor's action error (as test_gpu_policy)."""
    h = np.asarray(obs, np.float64)
    dh = U_BF16 * np.abs(h)
    for layer, (w, b) in enumerate(zip(ws, bs)):
        w = np.asarray(w, np.float64)
        aw = np.abs(w)
        dz = dh @ aw + (U_BF16 + w.shape[0] * 2.0 ** -24) * (np.abs(h) @ aw) + 1e-6
        h = np.tanh(h @ w + b)
        dh = dz + (U_BF16 * np.abs(h) if layer < len(ws) - 1 else 0.0)
    return dh * np.array([0.2, 0.1])


def _closed_loop_checked(pol, ws, bs, p, st, steps, sample, seed):
    """Plain env + policy closed loop; every step checked against the oracle on
    `sample` agents (all when None).  Returns the FP64 returns."""
    n = p.n_agents
    env = flock.Env(flock.Params(n_agents=n, box=p.box, sectors=p.sectors,
                                 flags=flock.ENV_FLAG_COUNTS))
    env.set_state(*[torch.from_numpy(a).cuda() for a in st])
    obs = env.reset()
    g = np.random.default_rng(seed)
    for t in range(steps):
        act = pol.forward(obs)
        torch.cuda.synchronize()
        o_h, a_h = obs.cpu().numpy(), act.cpu().numpy()
        rows = np.arange(n) if sample is None else np.sort(g.choice(n, sample, replace=False))
        ref = oracle.policy_forward(o_h[rows], ws, bs)
        err = np.abs(a_h[rows].astype(np.float64) - ref)
        assert (err <= _act_bound(o_h[rows], ws, bs)).all(), f"step {t}: action error {err.max()}"
        pre = tuple(a.cpu().numpy() for a in env.get_state())
        obs, rew = env.step(act)
        torch.cuda.synchronize()
        post = tuple(a.cpu().numpy() for a in env.get_state())
        check_move(post, oracle.oracle_move(pre, a_h, p.box), p.box, f"served n={n} step {t}")
        agents = None if sample is None else rows.astype(np.int32)
        o = oracle.oracle_sense(post[0], post[1], post[2], p.box, sectors=p.sectors,
                                agents=agents, eps_d=EPS_D, eps_phi=EPS_PHI)
        nb, col = (a.cpu().numpy() for a in env.counts())
        sel = slice(None) if agents is None else agents
        check_sense(o, obs.cpu().numpy()[sel], rew.cpu().numpy()[sel], nb[sel], col[sel],
                    label=f"served n={n} step {t}")
    torch.cuda.synchronize()
    return env.returns().cpu().numpy()


def test_served_mix_against_oracle_teacher_forced():
    """A 40,000-agent request served in a mix that arrives over several ticks
    (1,500 and 7,000 agents join while it runs): each request's FP64 returns
    equal the plain closed loop's bitwise, and that loop matches the oracle at
    every step (all agents of the small requests, 1,500 sampled agents of the
    large one)."""
    ws, bs = workloads.xavier_weights([16, 64, 64, 2], seed=0)
    bs = [b + np.float32(0.02) * (k + 1) for k, b in enumerate(bs)]
    pol = flock.Policy(ws, bs)
    reqs = [(request(40000, seed=61), 5), (request(1500, seed=62), 7), (request(7000, seed=63), 4)]
    srv = flock.Server(pol, 2 << 30, max_slots=8)
    ids = [srv.submit(reqs[0][0][0], reqs[0][0][1], steps=reqs[0][1])[0]]
    srv.tick()
    ids.append(srv.submit(reqs[1][0][0], reqs[1][0][1], steps=reqs[1][1])[0])
    srv.tick()
    ids.append(srv.submit(reqs[2][0][0], reqs[2][0][1], steps=reqs[2][1])[0])
    res, seen = drain(srv, ids)
    assert max(seen) == 3, "requests did not overlap"
    for rid, ((p, st), steps), sample, seed in zip(ids, reqs, (1500, None, None), (1, 2, 3)):
        ret = _closed_loop_checked(pol, ws, bs, p, st, steps, sample, seed)
        assert np.array_equal(res[rid], ret), f"request of {p.n_agents} agents"


def test_waiting_head_is_not_passed_over_forever():
    """A large request that cannot run beside the small ones keeps arriving
    behind it: after 32 ticks at the head of the queue it stops being passed
    over, the small ones drain, and it is admitted and finishes."""
    pol = policy()
    big = request(20000, seed=71)
    small_bytes = flock.request_bytes(request(500, seed=0)[0])
    srv = flock.Server(pol, flock.request_bytes(big[0]) + small_bytes // 2, max_slots=16)
    ids = [srv.submit(*request(500, seed=72), steps=10)[0]]
    bid, admitted = srv.submit(big[0], big[1], steps=3)
    assert not admitted
    for k in range(80):
        ids.append(srv.submit(*request(500, seed=100 + k), steps=10)[0])
        srv.tick()
        if srv.poll(bid)[0] == srv.FINISHED:
            break
    assert srv.poll(bid)[0] == srv.FINISHED, "the large request was passed over indefinitely"
    assert k >= 32
    res, _ = drain(srv, ids)
    assert len(res) == len(ids)
