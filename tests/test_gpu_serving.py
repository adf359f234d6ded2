"""Serving loop: continuous batching with footprint admission (GPU).

The same request must give bitwise the same FP64 returns whether it runs
alone or overlapped with others (deterministic bursts force the overlap),
and the same as the plain env + policy closed loop.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import workloads

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
