#!/usr/bin/env python3
"""Throughput of the flock-environment step on one MI355X: batched vs plain.

Workload (the `value`): 200 independent 5,000-agent flock envs (periodic box
of side 316, vision 8, collision 0.5, 16 sectors, seeded uniform actions
turn in [-0.2, 0.2], dspeed in [-0.1, 0.1]) stepped together by one batched
step; K steps replayed from one captured HIP graph, actions resident in HBM,
timed with HIP events on the stream over five replays (the median is the
value).  A "step" is the whole step path: move + cell count, scan, scatter,
sweep (view, reward, FP64 return) for every agent of every env.

Also reported on the same JSON line:
  plain      one 5,000-agent env stepped alone (eager per-step latency)
  flock50k   the 50,000-agent clustered env (64 blobs) and a uniform 50,000-agent
             env, plain and batched x20
  policy     the closed-loop step with the policy fused into the view sweep
             against the policy launched separately before the step
  serving    Poisson arrivals at 20/s for 60 s, then a sweep of arrival rates
             up to saturation (p50/p99 tick latency, agent-steps/s per rate)
  roofline   the dominant kernel (the neighbour sweep): the step's algorithmic
             bytes (44 + 4v per agent-step) per launch over its average
             HIP-event duration, against HBM
  cpu_baseline  the CPU oracle on the host cores (and on one core) on a
             bounded sample

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
# FP32 vector issue: 256 CUs x 64 lanes x 2.4 GHz, one lane-op per lane per
# clock (157.3 TFLOP/s counts an FMA as 2 and packed FP32 as 2 more; packed
# FP32 is not generated here).
VALU_PEAK = 256 * 64 * 2.4e9
VALU_ISSUE_PEAK = 256 * 2.4e9   # wave64 VALU instructions per second (one per clock per CU)
OPS_PER_CANDIDATE = 12     # image shift, d^2, radius and self tests, counts
OPS_PER_NEIGHBOUR = 30     # bearing, sector, per-sector minimum
V = 16                     # sectors of the paper-scale workloads
STEP_BYTES = 44 + 4 * V    # algorithmic bytes per agent-step of the whole step
SWEEP_BYTES = 8 + 4 + 4 * V + 4 + 16   # per agent: position, heading, view, reward, FP64 return r/w


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def make_envs(flock, workloads, n, box, count, init, seed0, **params):
    envs = []
    import torch
    params = {"sectors": V, **params}
    for k in range(count):
        if init == "blobs":
            st = workloads.blob_state(n, box, seed=seed0 + k)
        else:
            st = workloads.uniform_state(n, box, seed=seed0 + k)
        env = flock.Env(flock.Params(n_agents=n, box=box, **params))
        env.set_state(*[torch.from_numpy(a).cuda() for a in st])
        env.reset()
        envs.append(env)
    return envs


def device_actions(G, K, seed, tag=False):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    a = torch.rand(K, G, 2, device="cuda", generator=g) * 2.0 - 1.0
    a[..., 0] *= 0.2
    if tag:   # tag actions set the speed: U[0, 2)
        a[..., 1] = (a[..., 1] + 1.0)
    else:
        a[..., 1] *= 0.1
    return a.contiguous()


def bench_batched(flock, batch, K, W, seed, timed_reps=20, tag=False, reps=5):
    """Graph-replayed K-step runs (median of `reps`, HIP events on the stream),
    graph-replayed one-step latencies, and per-phase timing; returns a dict."""
    import torch
    G = batch.n
    act = device_actions(G, K, seed, tag)
    obs = torch.empty(G, batch.d, device="cuda")
    rew = torch.empty(K, G, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for t in range(W):
            batch.step(act[t % K], obs, rew[t % K], stream)
        # per-phase durations of eager steps, and the cost of an event bracket
        # with nothing inside it (two markers back to back on the idle stream),
        # which each phase's event pair adds to its kernel
        phases, empty = [], []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for t in range(timed_reps):
            phases.append(batch.step_timed(act[t % K], obs, rew[t % K], stream))
            e0.record(stream)
            e1.record(stream)
            e1.synchronize()
            empty.append(e0.elapsed_time(e1))
        # per-step latency: a one-step graph replayed K times, each replay
        # bracketed by events (back to back on the stream)
        for _ in range(2):      # capture and launch both starting tables' graphs
            batch.run(1, act[:1], obs, rew[:1], stream)
        ev1 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(K)]
        for t in range(K):
            ev1[t][0].record(stream)
            batch.run(1, act[:1], obs, rew[:1], stream)
            ev1[t][1].record(stream)
        stream.synchronize()
        lat = [a.elapsed_time(b) for a, b in ev1]
        # throughput: the K-step graph replayed `reps` times
        for _ in range(2):      # both starting tables (K odd alternates them)
            batch.run(K, act, obs, rew, stream)
        evk = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(reps):
            evk[r][0].record(stream)
            batch.run(K, act, obs, rew, stream)
            evk[r][1].record(stream)
        stream.synchronize()
        wall = time.perf_counter() - t0
    assert torch.isfinite(obs).all() and torch.isfinite(rew).all()
    runs_ms = [a.elapsed_time(b) for a, b in evk]
    el = float(np.median(runs_ms)) * 1e-3
    ph = np.mean(np.asarray(phases), axis=0)
    return {"agent_steps_per_s": G * K / el, "ms_per_step": 1e3 * el / K, "agents": G,
            "replay_ms": runs_ms, "replays_wall_s": wall,
            "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
            "latency_kind": "one-step graph replays, HIP events",
            "phase_ms": {"move_count": float(ph[0]), "scan": float(ph[1]),
                         "scatter": float(ph[2]), "sweep": float(ph[3])},
            "empty_bracket_ms": float(np.mean(empty)),
            "one_kernel_sort": bool(ph[1] == 0 and ph[2] == 0)}


def bench_plain(env, n, K, W, seed, tag=False):
    import torch
    act = device_actions(n, K, seed, tag)
    obs = torch.empty(n, env.d, device="cuda")
    rew = torch.empty(n, device="cuda")
    for t in range(W):
        env.step(act[t % K], obs, rew)
    torch.cuda.synchronize()
    # throughput: K back-to-back steps
    t0 = time.perf_counter()
    for t in range(K):
        env.step(act[t], obs, rew)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # latency: each step bracketed by events
    lat = []
    for t in range(K):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        env.step(act[t], obs, rew)
        e1.record()
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    return {"agent_steps_per_s": n * K / el, "ms_per_step": 1e3 * el / K, "agents": n,
            "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
            "latency_kind": "eager env_step calls, HIP events"}


def _serve(flock, pol, arrivals, sizes, boxes, states, steps, max_slots=64, arena=8 << 30):
    """Replay `arrivals` (seconds) in real time against one server; one tick per loop."""
    srv = flock.Server(pol, arena, max_slots=max_slots)
    ids, lat, agents, ticks, max_run, run_sum = [], [], 0, 0, 0, 0
    i, t0, busy = 0, time.perf_counter(), 0.0
    while True:
        now = time.perf_counter() - t0
        while i < len(arrivals) and arrivals[i] <= now:
            p = flock.Params(n_agents=int(sizes[i]), box=float(boxes[i]), sectors=V)
            ids.append(srv.submit(p, states[i], steps)[0])
            i += 1
        ts = time.perf_counter()
        n_run, ag = srv.tick()
        te = time.perf_counter()
        if n_run:
            lat.append(te - ts)
            busy += te - ts
            agents += ag
            ticks += 1
            run_sum += n_run
            max_run = max(max_run, n_run)
        elif i == len(arrivals):
            if all(srv.poll(r)[0] == srv.FINISHED for r in ids):
                break
        else:
            time.sleep(max(0.0, min(0.002, arrivals[i] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    for r in ids:
        srv.result(r)
    return {"requests": len(ids), "ticks": ticks, "max_running": max_run,
            "mean_running": run_sum / ticks if ticks else 0.0,
            "p50_ms": 1e3 * percentile(lat, 50) if lat else 0.0,
            "p99_ms": 1e3 * percentile(lat, 99) if lat else 0.0,
            "agent_steps_per_s_busy": agents / busy if busy else 0.0,
            "agent_steps_per_s_wall": agents / wall, "wall_s": wall,
            "offered_agent_steps_per_s": float(np.sum(sizes)) * steps / max(arrivals[-1], 1e-9)
            if len(arrivals) else 0.0}


def bench_serving(flock, workloads, duration=60.0, rates=(20, 100, 500, 2000, 5000), lo=500,
                  hi=50000, steps=200, seed=0, max_requests=2000, window=4.0):
    """Serving loop (continuous batching, fused BF16 policy): Poisson arrivals
    of episode requests, one closed-loop step per tick over every running
    request; the tick (= step) latency is the host wall time of srv_tick, which
    ends with a stream synchronisation.

    First `duration` seconds of arrivals at rates[0]/s; then each rate of
    `rates` for min(window, max_requests / rate) seconds of arrivals, drained,
    stopping after the first rate whose p99 tick latency exceeds twice its p50.
    """
    ws, bs = workloads.xavier_weights([V, 64, 64, 2], seed=0)
    pol = flock.Policy(ws, bs)

    def point(rate, dur, seed_k):
        arrivals = workloads.poisson_arrivals(rate, dur, seed_k)[:max_requests]
        sizes, boxes = workloads.uneven_env_sizes(len(arrivals), lo, hi, seed=seed_k + 1)
        states = [workloads.uniform_state(int(n), float(b), seed=seed_k, env=k)
                  for k, (n, b) in enumerate(zip(sizes, boxes))]
        res = _serve(flock, pol, arrivals, sizes, boxes, states, steps)
        res.update({"rate_per_s": rate, "arrival_s": float(dur),
                    "largest_request": int(np.max(sizes)) if len(sizes) else 0})
        return res

    log(f"[bench] serving: Poisson {rates[0]}/s for {duration} s")
    long_run = point(rates[0], duration, seed)
    sweep = []
    for k, rate in enumerate(rates):
        dur = min(window, max_requests / rate)
        log(f"[bench] serving: rate {rate}/s for {dur:.2f} s")
        r = point(rate, dur, seed + 100 * (k + 1))
        sweep.append(r)
        if r["p99_ms"] > 2.0 * r["p50_ms"]:
            break
    return {"workload": f"Poisson arrivals, N log-uniform [{lo}, {hi}], side 4 sqrt(N), 16 "
                        f"sectors, {steps} steps each, fused BF16 policy, at most 64 running",
            "poisson": {**long_run, "rate_per_s": rates[0], "arrival_s": duration},
            "rate_sweep": sweep}


def bench_policy(flock, workloads, envs, K, W):
    """Closed-loop step (env_step_policy) over the 200 x 5,000-agent batch:
    the policy as its own launch before the step (the default) against the
    policy run inside the view sweep (policy fusion on).  Eager calls, HIP
    events over K steps each."""
    import torch
    batch = flock.Batch(envs)
    fused_batch = flock.Batch(envs)
    fused_batch.set_policy_fusion(True)
    G = batch.n
    ws, bs = workloads.xavier_weights([V, 64, 64, 2], seed=0)
    pol = flock.Policy(ws, bs)
    obs = torch.empty(G, V, device="cuda")
    act = torch.zeros(G, 2, device="cuda")
    rew = torch.empty(G, device="cuda")
    stream = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    with torch.cuda.stream(stream):
        batch.step(act, obs, rew, stream)         # a current view
        for _ in range(W):
            fused_batch.step_policy(pol, act, obs, rew, stream)
        ev[0].record(stream)
        for _ in range(K):
            fused_batch.step_policy(pol, act, obs, rew, stream)
        ev[1].record(stream)
        for _ in range(W):
            batch.step_policy(pol, act, obs, rew, stream)
        ev[2].record(stream)
        for _ in range(K):
            batch.step_policy(pol, act, obs, rew, stream)
        ev[3].record(stream)
        for _ in range(K):
            pol.forward(obs, act, stream)
        ev[4].record(stream)
        stream.synchronize()
    assert torch.isfinite(obs).all() and torch.isfinite(act).all()
    fused = ev[0].elapsed_time(ev[1]) / K
    separate = ev[2].elapsed_time(ev[3]) / K
    pol_ms = ev[3].elapsed_time(ev[4]) / K
    flop = 2 * G * (V * 64 + 64 * 64 + 64 * 2)
    return {"workload": f"{len(envs)} envs x 5,000 agents, closed loop, 16 -> 64 -> 64 -> 2 "
                        "BF16 policy (MFMA 16x16x32, FP32 accumulate)",
            "agents": G, "fused_ms_per_step": fused, "separate_ms_per_step": separate,
            "policy_kernel_ms": pol_ms, "fused_agent_steps_per_s": G / (fused * 1e-3),
            "separate_agent_steps_per_s": G / (separate * 1e-3),
            "mlp_flop_per_step": flop,
            "policy_kernel_mfma_frac": flop / (pol_ms * 1e-3) / 2.5e15}


def bench_rollout(flock, workloads, reps=3):
    """Experience collection of one training step (Sec. 5: t = 128 updates).

    One env with the paper's flock settings at 16,000 agents; 128 sampled
    closed-loop steps written into the rollout buffers (env_rollout, one HIP
    graph), the critic over all 129 x 16,000 views, then the advantages.
    """
    import torch
    from paper_2207_03945_amd import autotune
    pf = workloads.WORKLOADS["paper_flock10k"]
    n, T = 16000, 128
    kw = dict(n_agents=n, box=pf["box"], radius=pf["radius"], sectors=pf["sectors"],
              fov=math.radians(pf["fov_deg"]), flags=flock.ENV_FLAG_SPEED_OBS)
    state = workloads.uniform_state(n, pf["box"], seed=77)
    # cell reach and sweep lanes timed on this env (one dense env: wide lane groups)
    reach, lanes, tuned = autotune.tune([flock.Params(**kw)], [state], cache=None)
    p = flock.Params(cell_reach=reach, **kw)
    env = flock.Env(p)
    env.set_state(*[torch.from_numpy(a).cuda() for a in state])
    obs0 = env.reset()
    b = flock.Batch([env])
    b.set_sweep_lanes(lanes)
    d = p.obs_dim
    aw, ab = workloads.xavier_weights([d, 64, 64, 2], seed=1)
    cw, cb = workloads.xavier_weights([d, 64, 64, 1], seed=2)
    pol, cri = flock.Policy(aw, ab), flock.Critic(cw, cb)
    obs = torch.empty(T + 1, n, d, device="cuda")
    act = torch.empty(T, n, 2, device="cuda")
    logp = torch.empty(T, n, device="cuda")
    rew = torch.empty(T, n, device="cuda")
    val = torch.empty(T + 1, n, device="cuda")
    adv = torch.empty(T, n, device="cuda")
    ret = torch.empty(T, n, device="cuda")
    eps = torch.from_numpy(workloads.policy_noise(T, n, seed=3)).cuda()
    log_std = (-1.6, -2.3)
    stream = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    times = []
    with torch.cuda.stream(stream):
        obs[0].copy_(obs0)
        for rep in range(reps + 1):
            ev[0].record(stream)
            b.rollout(pol, T, obs, act, rew, logp=logp, eps=eps, log_std=log_std, stream=stream)
            ev[1].record(stream)
            cri.value(obs, out=val, stream=stream)
            ev[2].record(stream)
            flock.gae(rew, val, 0.99, 0.95, adv=adv, ret=ret, stream=stream)
            ev[3].record(stream)
            obs[0].copy_(obs[T])
            stream.synchronize()
            if rep:   # the first pass captures the graph
                times.append([ev[k].elapsed_time(ev[k + 1]) for k in range(3)])
    assert torch.isfinite(adv).all() and torch.isfinite(val).all()
    t = np.median(np.asarray(times), axis=0)
    gae_bytes = 16 * T * n
    # critic FLOPs over the (T + 1) n views: in x 64 + 64 x 64 + 64 x 1 MACs per row
    critic_flop = 2 * (T + 1) * n * (d * 64 + 64 * 64 + 64)
    critic_bytes = (T + 1) * n * (4 * d + 4)
    return {"workload": f"one env, {n:,} agents, the paper's flock settings (box 100, vision 10, "
                        f"128 sectors, 250 degrees, speed in the view), {T} sampled steps per "
                        "collection; critic over the 129 x N views; advantages",
            "cell_reach": reach, "sweep_lanes": lanes, "tuned_ms": tuned,
            "rollout_ms": float(t[0]), "critic_ms": float(t[1]), "gae_ms": float(t[2]),
            "collect_ms": float(t.sum()), "agent_steps_per_s": n * T / (t[0] * 1e-3),
            "buffer_bytes": int((obs.numel() + act.numel() + logp.numel() + rew.numel()
                                 + val.numel() + adv.numel() + ret.numel()) * 4),
            "critic_mfma": {"flop_per_launch": critic_flop,
                            "achieved_TFLOPs": critic_flop / (t[1] * 1e-3) / 1e12,
                            "peak_TFLOPs": 2500.0,
                            "frac": critic_flop / (t[1] * 1e-3) / 2.5e15},
            # the critic's bound is reading the FP32 views (+ 4 B out per row)
            "critic_hbm": {"bytes_per_launch": critic_bytes,
                           "achieved_GBps": critic_bytes / (t[1] * 1e-3) / 1e9,
                           "frac": critic_bytes / (t[1] * 1e-3) / HBM_PEAK},
            "gae_hbm": {"bytes_per_launch": gae_bytes,
                        "achieved_GBps": gae_bytes / (t[2] * 1e-3) / 1e9,
                        "frac": gae_bytes / (t[2] * 1e-3) / HBM_PEAK}}


def bench_graph(flock, workloads, steps=50):
    """Opinion dynamics over a 1,000,000-node power-law social graph (Sec. 2.1)."""
    import torch
    n = 1_000_000
    rp, col, w = workloads.social_graph(n, seed=0)
    E = int(rp[-1])
    rp_d = torch.from_numpy(rp).cuda()
    col_d = torch.from_numpy(col).cuda()
    w_d = torch.from_numpy(w).cuda()
    a = torch.from_numpy(workloads.opinions(n, seed=0)).cuda()
    b = torch.empty_like(a)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    res = {}
    for lanes in (1, 4, 16):
        for _ in range(3):
            flock.opinion_step(rp_d, col_d, w_d, a, b, 0.3, 0.5, lanes=lanes)
            a, b = b, a
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(steps):
            flock.opinion_step(rp_d, col_d, w_d, a, b, 0.3, 0.5, lanes=lanes)
            a, b = b, a
        ev[1].record()
        ev[1].synchronize()
        res[lanes] = ev[0].elapsed_time(ev[1]) / steps
    best = min(res, key=res.get)
    ms = res[best]
    algo = 16 * n + 12 * E
    return {"workload": f"{n:,} nodes, {E:,} directed edges (power-law degrees 5..2,000), "
                        "threshold 0.3, strength 0.5",
            "ms_per_step_by_lanes": {str(k): v for k, v in res.items()}, "lanes": best,
            "ms_per_step": ms, "edges_per_s": E / (ms * 1e-3),
            "hbm": {"algorithmic_bytes_per_step": algo, "achieved_GBps": algo / (ms * 1e-3) / 1e9,
                    "frac": algo / (ms * 1e-3) / HBM_PEAK}}


def cpu_baseline_inproc(seconds):
    """The oracle (all-pairs, FP64 view) on the host, 5,000-agent env, bounded sample."""
    import oracle
    import workloads
    oracle.build()
    n, box = 5000, 316.0
    st = workloads.uniform_state(n, box, seed=0)
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and steps < 1000:
        act = workloads.random_actions(n, seed=0, step=steps)
        st, _ = oracle.oracle_step(st, act, box, sectors=V)
        steps += 1
    el = time.perf_counter() - t0
    return {"value": n * steps / el, "unit": "agent-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one 5,000-agent env (side 316, 16 sectors), first {steps} steps "
                      f"(move + all-pairs view/reward), {el:.1f} s"}


def cpu_baseline(seconds):
    """The oracle timed in child processes (before this process touches the
    GPU): on every host core, then on one."""
    import subprocess
    out = {}
    for label, threads in (("all", None), ("one", 1)):
        env = dict(os.environ)
        if threads:
            env["OMP_NUM_THREADS"] = str(threads)
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                            str(seconds)], env=env, capture_output=True, text=True, check=True)
        out[label] = json.loads(r.stdout.strip().splitlines()[-1])
    res = dict(out["all"])
    res["single_thread"] = out["one"]
    return res


def sweep_work(envs, radius=8.0):
    """Candidate tests and neighbour pairs of one sweep over these envs' current states.

    Candidates are those of the textbook cell list, independent of the grid
    the kernels use: for each agent, every agent of the 3 x 3 block of square
    cells of side at least the vision range round its own (itself included;
    all n when fewer than 3 such cells fit the side).  Neighbours: ordered
    pairs closer than the vision range (periodic k-d tree).
    """
    from scipy.spatial import cKDTree
    cand = nbrs = 0
    for e in envs:
        x, y = (t.cpu().numpy().astype(np.float64) for t in e.get_state()[:2])
        n = x.shape[0]
        if n == 0:
            continue
        box = e.params.box
        nc, reach = int(box // e.params.radius), 1
        if nc < 3:
            cand += n * n
        else:
            cx = np.minimum((x * (nc / box)).astype(np.int64), nc - 1)
            cy = np.minimum((y * (nc / box)).astype(np.int64), nc - 1)
            grid = np.zeros((nc, nc), np.int64)
            np.add.at(grid, (cx, cy), 1)
            block = np.zeros_like(grid)
            for dx in range(-reach, reach + 1):
                for dy in range(-reach, reach + 1):
                    block += np.roll(np.roll(grid, dx, 0), dy, 1)
            cand += int(block[cx, cy].sum())
        pts = np.stack([np.mod(x, box), np.mod(y, box)], 1)
        tree = cKDTree(pts, boxsize=box)
        nbrs += int(tree.count_neighbors(tree, e.params.radius)) - n
    return {"candidates": cand, "neighbours": nbrs,
            "lane_ops": OPS_PER_CANDIDATE * cand + OPS_PER_NEIGHBOUR * nbrs}


def alu_roofline(work, sweep_ms):
    """The textbook cell list's modelled lane operations over the sweep's time:
    an upper reference, not a bound (the kernel tests fewer candidates than
    the textbook 3 x 3 block, so this can exceed the issue peak)."""
    achieved = work["lane_ops"] / (sweep_ms * 1e-3)
    return {"modelled_T_lane_ops": achieved / 1e12, "issue_peak_T": VALU_PEAK / 1e12}


def sweep_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2207_03945_amd", "csrc", "flock_kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def profile_record(agents):
    """The committed PMC summary of the main leg's sweep (HBM bytes and VALU
    instructions per launch), if it was taken from the current kernel source."""
    path = os.path.join(ROOT, "profiles", "sweep_flock5k_x200_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != sweep_source_hash() or t.get("agents") != agents:
        return None
    return t


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--envs", type=int, default=200, help="5,000-agent envs in the batch")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-main", action="store_true", help="run the main batched leg only")
    ap.add_argument("--legs", default="plain,policy,50k,uneven,rollout,graph,serving",
                    help="comma list of extra legs: plain, policy, 50k, uneven, paper, tag, "
                         "rollout, graph, serving (paper and tag, the paper-scale flock and "
                         "tag batches, only when asked for)")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--cpu-baseline-child", type=float, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.cpu_baseline_child is not None:
        print(json.dumps(cpu_baseline_inproc(args.cpu_baseline_child)), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the flock step has no multi-GPU path "
              "(independent envs would shard across GPUs with no communication); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (before the GPU is used)")
        cpu = cpu_baseline(args.cpu_seconds)

    import torch

    import paper_2207_03945_amd as flock
    import workloads
    from paper_2207_03945_amd import autotune

    flock.lib()
    K, W = args.steps, args.warmup
    torch.cuda.init()

    log(f"[bench] batched 5k x {args.envs}")
    envs = make_envs(flock, workloads, 5000, 316.0, args.envs, "uniform", 1000)
    batch = flock.Batch(envs)
    torch.cuda.synchronize()
    # barrier + synchronize bracket the timed region inside bench_batched
    main_res = bench_batched(flock, batch, K, W, seed=1)
    main_res["sweep_lanes"] = batch.sweep_lanes
    G = batch.n
    del batch
    main_work = sweep_work(envs)
    extra = {}
    legs = set() if args.only_main else {x for x in args.legs.split(",") if x}
    if "plain" in legs:
        log("[bench] plain 5k")
        extra["plain"] = bench_plain(envs[0], 5000, K, W, seed=2)
    if "policy" in legs:
        log("[bench] closed loop with the fused policy")
        extra["policy"] = bench_policy(flock, workloads, envs, min(K, 100), W)
    del envs
    if "50k" in legs:
        for name, init in (("blobs50k", "blobs"), ("uniform50k", "uniform")):
            log(f"[bench] {name} plain")
            e50 = make_envs(flock, workloads, 50000, 1000.0, 20, init, 2000)
            plain = bench_plain(e50[0], 50000, K, W, seed=3)
            log(f"[bench] {name} batched x20")
            b50 = flock.Batch(e50)
            lane_ms = autotune.time_sweep_lanes(b50, (1, 4, 16))
            b50.set_sweep_lanes(min(lane_ms, key=lane_ms.get))
            bat = bench_batched(flock, b50, K, W, seed=4, timed_reps=10)
            extra[name] = {"plain": plain, "batched_x20": {**bat, "sweep_lanes": b50.sweep_lanes,
                                                           "lanes_ms": lane_ms}}
            del b50, e50
    if "uneven" in legs:
        log("[bench] uneven 256 envs")
        ns, boxes = workloads.uneven_env_sizes(256, 100, 20000, seed=0)
        states = [workloads.uniform_state(int(n), float(b), seed=0, env=k)
                  for k, (n, b) in enumerate(zip(ns, boxes))]
        plist = [flock.Params(n_agents=int(n), box=float(b), sectors=V) for n, b in zip(ns, boxes)]
        reach, lanes, tune_ms = autotune.tune(plist, states, cache=None)
        envs_u = []
        for p_, st in zip(plist, states):
            p_.cell_reach = reach
            e = flock.Env(p_)
            e.set_state(*[torch.from_numpy(a).cuda() for a in st])
            e.reset()
            envs_u.append(e)
        bu = flock.Batch(envs_u)
        bu.set_sweep_lanes(lanes)
        extra["uneven256"] = {"agents": bu.n, "cell_reach": reach, "sweep_lanes": lanes,
                              "tuned_ms": tune_ms,
                              **bench_batched(flock, bu, K, W, seed=5, timed_reps=10)}
        del bu, envs_u
    if "paper" in legs:
        log("[bench] paper flock 10k")
        pf = workloads.WORKLOADS["paper_flock10k"]
        pf_params = dict(sectors=pf["sectors"], radius=pf["radius"],
                         fov=math.radians(pf["fov_deg"]), flags=flock.ENV_FLAG_SPEED_OBS)
        pf_plist = [flock.Params(n_agents=pf["n"], box=pf["box"], **pf_params) for _ in range(20)]
        pf_states = [workloads.uniform_state(pf["n"], pf["box"], seed=3000 + k) for k in range(20)]
        pf_reach, pf_lanes, pf_ms = autotune.tune(pf_plist, pf_states, cache=None)
        e10 = make_envs(flock, workloads, pf["n"], pf["box"], 20, "uniform", 3000,
                        cell_reach=pf_reach, **pf_params)
        e10[0].set_sweep_lanes(pf_lanes)
        plain = bench_plain(e10[0], pf["n"], K, W, seed=6)
        b10 = flock.Batch(e10)
        b10.set_sweep_lanes(pf_lanes)
        bat = bench_batched(flock, b10, K, W, seed=7, timed_reps=10)
        work = sweep_work(e10)
        pf_bytes = 8 + 4 + 4 * (pf["sectors"] + 1) + 4 + 16
        extra["paper_flock10k"] = {
            "workload": "20 envs x 10,000 agents, side 100, vision 10 (L/10), 128 sectors, "
                        "field of view 250 degrees, speed appended (129 values)",
            "cell_reach": pf_reach, "sweep_lanes": pf_lanes, "tuned_ms": pf_ms,
            "plain": plain, "batched_x20": bat, "sweep_work_per_launch": work,
            "sweep_valu_lane_ops_model": alu_roofline(work, bat["phase_ms"]["sweep"]),
            "sweep_hbm_frac": pf_bytes * b10.n / (bat["phase_ms"]["sweep"] * 1e-3) / HBM_PEAK}
        del b10, e10
    if "tag" in legs:
        log("[bench] tag 11k")
        tg = workloads.WORKLOADS["paper_tag11k"]
        tg_params = dict(sectors=tg["sectors"], radius=tg["radius"], collide=tg["touch"],
                         fov=math.radians(tg["fov_deg"]), flags=flock.ENV_FLAG_TAG,
                         n_chasers=tg["chasers"], r_catch=1.0)
        tg_plist = [flock.Params(n_agents=tg["n"], box=tg["box"], **tg_params) for _ in range(20)]
        tg_states = [workloads.uniform_state(tg["n"], tg["box"], seed=4000 + k) for k in range(20)]
        tg_reach, tg_lanes, tg_ms = autotune.tune(tg_plist, tg_states, cache=None)
        e11 = make_envs(flock, workloads, tg["n"], tg["box"], 20, "uniform", 4000,
                        cell_reach=tg_reach, **tg_params)
        e11[0].set_sweep_lanes(tg_lanes)
        plain = bench_plain(e11[0], tg["n"], K, W, seed=8, tag=True)
        b11 = flock.Batch(e11)
        b11.set_sweep_lanes(tg_lanes)
        bat = bench_batched(flock, b11, K, W, seed=9, timed_reps=10, tag=True)
        work = sweep_work(e11)
        extra["paper_tag11k"] = {
            "workload": "20 envs x 11,000 agents (1,000 chasers), side 100, vision 10, two "
                        "channels of 64 sectors, field of view 250 degrees, touch distance 1",
            "cell_reach": tg_reach, "sweep_lanes": tg_lanes, "tuned_ms": tg_ms,
            "plain": plain, "batched_x20": bat, "sweep_work_per_launch": work,
            "sweep_valu_lane_ops_model": alu_roofline(work, bat["phase_ms"]["sweep"])}
        del b11, e11
    if "rollout" in legs:
        log("[bench] experience collection")
        extra["rollout"] = bench_rollout(flock, workloads)
    if "graph" in legs:
        log("[bench] graph interaction")
        extra["graph"] = bench_graph(flock, workloads)
    if "serving" in legs:
        log("[bench] serving")
        extra["serving"] = bench_serving(flock, workloads, duration=args.serve_seconds)

    if args.copy_calib_mib:
        src = torch.ones(args.copy_calib_mib << 18, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # Roofline of the dominant kernel (the neighbour sweep) against HBM: the
    # step's algorithmic bytes, 44 + 4v per agent-step (read x, y, heading,
    # speed and the action; write the state, the view and the reward), times
    # the agents one launch covers, over the launch's average duration: HIP
    # events around it on its stream (eager steps), less the measured cost of
    # an empty event bracket.  The sweep is bound by vector issue in practice;
    # the committed PMC record gives that fraction when current.
    sweep_event_ms = main_res["phase_ms"]["sweep"]
    sweep_ms = sweep_event_ms - main_res["empty_bracket_ms"]
    if not sweep_ms > 0.0:
        sweep_ms = sweep_event_ms
    algo = STEP_BYTES * G
    achieved = algo / (sweep_ms * 1e-3)
    prof = profile_record(G)
    traffic = prof.get("bytes_per_launch") if prof else None
    roofline = {"kernel": "k_sweep", "bound": "hbm", "achieved": achieved / 1e9,
                "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": achieved / HBM_PEAK,
                "traffic": traffic,
                "traffic_over_algorithmic": traffic / algo if traffic else None,
                "avg_launch_ms": sweep_ms, "avg_launch_event_ms": sweep_event_ms,
                "empty_bracket_ms": main_res["empty_bracket_ms"],
                "algorithmic_bytes_per_launch": algo,
                "bytes_model": f"44 + 4v = {STEP_BYTES} B per agent-step x {G} agents",
                "step": {"achieved": STEP_BYTES * main_res["agent_steps_per_s"] / 1e9,
                         "frac": STEP_BYTES * main_res["agent_steps_per_s"] / HBM_PEAK},
                "valu_issue_frac": (prof["valu_insts_per_launch"] / (VALU_ISSUE_PEAK *
                                                                      sweep_ms * 1e-3))
                if prof and prof.get("valu_insts_per_launch") else None,
                "textbook_work": main_work}
    for name in ("blobs50k", "uniform50k"):
        if name in extra:
            b = extra[name]["batched_x20"]
            b["step_hbm_frac"] = STEP_BYTES * b["agent_steps_per_s"] / HBM_PEAK
            extra[name]["plain"]["step_hbm_frac"] = (STEP_BYTES *
                                                      extra[name]["plain"]["agent_steps_per_s"] /
                                                      HBM_PEAK)

    out = {
        "metric": "agent-steps/s batched vs plain at 5k/50k agents; p50/p99 step latency",
        "value": main_res["agent_steps_per_s"],
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"flock5k x{args.envs} batched: {args.envs} envs x 5,000 agents, "
                               "side 316, vision 8, 16 sectors, seeded uniform actions",
                   "envs": args.envs, "agents": G, "graph_steps": K},
        "batched": main_res,
        **extra,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
