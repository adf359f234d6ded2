"""Seeded synthetic inputs for the flock environment.

This module only draws random numbers of the right shapes and ranges; it holds
none of the environment's arithmetic, so both the CPU oracle and the GPU path
can consume its outputs.  Every stream is keyed by (seed, purpose, env, step)
through numpy's SeedSequence, so a given array does not depend on what else
was drawn before it.

Workloads (all FP32, periodic square box of side L):
  * uniform:  positions U[0, L)^2, headings U[0, 2pi), speed 1.0
  * blobs:    64 isotropic Gaussian blobs (sigma 6), centres U[0, L)^2,
              agent i in blob i mod 64, positions wrapped into the box
  * actions:  turn U[-0.2, 0.2] rad, dspeed U[-0.1, 0.1]
  * uneven env sizes: N_e = round(exp(U[ln lo, ln hi])), side L_e = 4 sqrt(N_e)
  * arrivals: Poisson process (exponential gaps) for the serving loop
  * policy noise: standard normals [steps, n, 2] for Gaussian action sampling
  * paper tag (Sec. 4.2, 5): a chaser per ten runners (agents 0 .. n/11 - 1
    chase), two view channels of 64 sectors, 250 degrees, vision L/10,
    touch distance 1; uniform start; speeds U[0, 2) as the action
  * social graph: power-law degrees (exponent 2.5, 5..2,000, mean about 14),
    configuration-model pairing, symmetric weights U[0, 1), opinions U[0, 1)
  * paper flock (Sec. 4.1, 5): v = 128 sectors, a field of view of 250
    degrees, the speed appended to the view (129 values), vision range one
    tenth of the box side; uniform start.  With R = L/10 the mean number of
    neighbours is pi N / 100 whatever L, so only N sets the density.
"""
from __future__ import annotations

import math

import numpy as np

PURPOSE_STATE = 1
PURPOSE_ACTION = 2
PURPOSE_WEIGHTS = 3
PURPOSE_SIZES = 4
PURPOSE_ARRIVALS = 5
PURPOSE_BLOB_CENTRES = 6
PURPOSE_POLICY_NOISE = 7
PURPOSE_GRAPH = 8


def rng(seed: int, purpose: int, env: int = 0, step: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [int(seed) & 0xFFFFFFFF, int(purpose), int(env), int(step)])))


def _into_box(v: np.ndarray, box: float) -> np.ndarray:
    """Round to FP32 and fold into [0, box): values that round up to box become 0."""
    f = np.mod(v, box).astype(np.float32)
    f[f >= np.float32(box)] = np.float32(0.0)
    f[f < 0] = np.float32(0.0)
    return f


def _headings(g: np.random.Generator, n: int) -> np.ndarray:
    th = (g.random(n) * (2.0 * math.pi)).astype(np.float32)
    th[th >= np.float32(2.0 * math.pi)] = np.float32(0.0)
    return th


def uniform_state(n: int, box: float, seed: int = 0, env: int = 0, speed: float = 1.0):
    """(x, y, th, s) FP32 arrays for n agents uniform in the box."""
    g = rng(seed, PURPOSE_STATE, env)
    x = _into_box(g.random(n) * box, box)
    y = _into_box(g.random(n) * box, box)
    th = _headings(g, n)
    s = np.full(n, speed, np.float32)
    return x, y, th, s


def blob_state(n: int, box: float, seed: int = 0, env: int = 0, n_blobs: int = 64,
               sigma: float = 6.0, speed: float = 1.0):
    """(x, y, th, s) for n agents in n_blobs Gaussian blobs (agent i -> blob i mod n_blobs)."""
    gc = rng(seed, PURPOSE_BLOB_CENTRES, env)
    centres = gc.random((n_blobs, 2)) * box
    g = rng(seed, PURPOSE_STATE, env)
    blob = np.arange(n) % n_blobs
    offs = g.normal(0.0, sigma, (n, 2))
    x = _into_box(centres[blob, 0] + offs[:, 0], box)
    y = _into_box(centres[blob, 1] + offs[:, 1], box)
    th = _headings(g, n)
    s = np.full(n, speed, np.float32)
    return x, y, th, s


def tag_actions(n: int, seed: int = 0, step: int = 0, env: int = 0, max_turn: float = 0.2,
                s_max: float = 2.0) -> np.ndarray:
    """Tag actions [n, 2] FP32: turn U[-max_turn, max_turn], speed U[0, s_max)."""
    g = rng(seed, PURPOSE_ACTION, env, step)
    a = g.random((n, 2))
    return np.stack([(2.0 * a[:, 0] - 1.0) * max_turn, a[:, 1] * s_max], 1).astype(np.float32)


def random_actions(n: int, seed: int = 0, step: int = 0, env: int = 0,
                   max_turn: float = 0.2, max_dspeed: float = 0.1) -> np.ndarray:
    """[n, 2] FP32 actions: column 0 = turn, column 1 = dspeed."""
    g = rng(seed, PURPOSE_ACTION, env, step)
    a = np.empty((n, 2), np.float32)
    a[:, 0] = (g.random(n) * 2.0 - 1.0) * max_turn
    a[:, 1] = (g.random(n) * 2.0 - 1.0) * max_dspeed
    return a


def uneven_env_sizes(n_envs: int, lo: int, hi: int, seed: int = 0):
    """Log-uniform agent counts in [lo, hi] and box sides 4 sqrt(N) (density 1/16)."""
    g = rng(seed, PURPOSE_SIZES)
    n = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), n_envs))).astype(np.int64)
    n = np.clip(n, lo, hi)
    box = np.array([float(np.float32(4.0 * math.sqrt(k))) for k in n])
    return n, box


def xavier_weights(dims, seed: int = 0):
    """Glorot-uniform FP32 weights (fan_in, fan_out) per layer and zero biases."""
    ws, bs = [], []
    for layer in range(len(dims) - 1):
        fi, fo = dims[layer], dims[layer + 1]
        a = math.sqrt(6.0 / (fi + fo))
        g = rng(seed, PURPOSE_WEIGHTS, layer)
        ws.append(((g.random((fi, fo)) * 2.0 - 1.0) * a).astype(np.float32))
        bs.append(np.zeros(fo, np.float32))
    return ws, bs


def policy_noise(steps: int, n: int, seed: int = 0, env: int = 0) -> np.ndarray:
    """Standard-normal draws [steps, n, 2] (FP32) for sampling actions round the policy mean."""
    g = rng(seed, PURPOSE_POLICY_NOISE, env)
    return g.standard_normal((steps, n, 2)).astype(np.float32)


def social_graph(n: int, seed: int = 0, k_min: int = 5, k_max: int = 2000, alpha: float = 2.5):
    """Undirected social graph as CSR of incoming edges, both directions stored.

    Degrees follow a discrete power law P(k) ~ k^-alpha on [k_min, k_max]
    (mean about 14 for the defaults); stubs are paired at random
    (configuration model), self loops dropped, repeated pairs kept.  Each
    undirected pair draws one weight U[0, 1) used by both directions.  Within
    a node's row, edges are in the order the pairing produced them.
    Returns (row_ptr int64 [n + 1], col int32 [E], weight float32 [E]).
    """
    g = rng(seed, PURPOSE_GRAPH)
    u = g.random(n)
    a1 = 1.0 - alpha
    k = (k_min ** a1 + u * (k_max ** a1 - k_min ** a1)) ** (1.0 / a1)
    deg = np.floor(k).astype(np.int64)
    stubs = np.repeat(np.arange(n, dtype=np.int64), deg)
    g.shuffle(stubs)
    m = stubs.shape[0] // 2
    a, b = stubs[:m], stubs[m:2 * m]
    keep = a != b
    a, b = a[keep], b[keep]
    w = g.random(a.shape[0]).astype(np.float32)
    me = np.concatenate([a, b])
    you = np.concatenate([b, a])
    ww = np.concatenate([w, w])
    order = np.argsort(me, kind="stable")
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(me, minlength=n), out=row_ptr[1:])
    return row_ptr, you[order].astype(np.int32), ww[order]


def opinions(n: int, seed: int = 0) -> np.ndarray:
    """Initial opinions U[0, 1), FP32."""
    return rng(seed, PURPOSE_GRAPH, 1).random(n).astype(np.float32)


def poisson_arrivals(rate: float, duration: float, seed: int = 0):
    """Arrival times (s) of a Poisson process of the given rate over [0, duration)."""
    g = rng(seed, PURPOSE_ARRIVALS)
    t, out = 0.0, []
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            return np.array(out)
        out.append(t)


# Named workloads (paper scale and stress cases) --------------------------------

WORKLOADS = {
    # 256 agents, 64 x 64 box, 8 sectors, 100 steps
    "flock256": dict(n=256, box=64.0, sectors=8, steps=100, init="uniform"),
    # 5,000 agents, side 316, 16 sectors, 1,000 steps
    "flock5k": dict(n=5000, box=316.0, sectors=16, steps=1000, init="uniform"),
    # 50,000 agents in 64 blobs, side 1,000, 16 sectors, 500 steps
    "blobs50k": dict(n=50000, box=1000.0, sectors=16, steps=500, init="blobs"),
    # 50,000 agents uniform, side 1,000 (control for the clustered case)
    "uniform50k": dict(n=50000, box=1000.0, sectors=16, steps=500, init="uniform"),
    # the paper's own flock settings at 1,000 and 10,000 agents (box 100, R 10)
    "paper_flock1k": dict(n=1000, box=100.0, radius=10.0, sectors=128, fov_deg=250.0,
                          speed_obs=True, steps=128, init="uniform"),
    "paper_flock10k": dict(n=10000, box=100.0, radius=10.0, sectors=128, fov_deg=250.0,
                           speed_obs=True, steps=128, init="uniform"),
    # the paper's tag settings: a chaser per ten runners, two channels of 64
    # sectors, 250 degrees, vision L/10, touch distance 1
    "paper_tag1k": dict(n=1100, chasers=100, box=100.0, radius=10.0, sectors=64, fov_deg=250.0,
                        touch=1.0, steps=128, init="uniform"),
    "paper_tag11k": dict(n=11000, chasers=1000, box=100.0, radius=10.0, sectors=64,
                         fov_deg=250.0, touch=1.0, steps=128, init="uniform"),
}


def make_state(name_or_cfg, seed: int = 0, env: int = 0):
    cfg = WORKLOADS[name_or_cfg] if isinstance(name_or_cfg, str) else name_or_cfg
    if cfg.get("init", "uniform") == "blobs":
        return blob_state(cfg["n"], cfg["box"], seed, env)
    return uniform_state(cfg["n"], cfg["box"], seed, env)
