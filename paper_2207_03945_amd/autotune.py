"""Autotuner for the batched step: cell reach and sweep lanes per agent.

Two launch choices change the speed of a step but never its result:

* the cell reach r of each env: cells at least R/r wide and a (2r + 1)^2
  block of cells per agent.  r = 1 tests fewer cells with more candidates
  each; r = 2 cuts candidates by about a third (25 R^2/4 vs 9 R^2 of area)
  at the price of more, shorter runs;
* the lanes per agent of the neighbour sweep (1, 4, 16 or 64): one lane per
  agent suits sparse neighbourhoods, a lane group per agent dense ones.

Which wins depends on the local density, the sector count and how the runs
fill the wavefronts, so it is measured: each candidate is timed on the
caller's own batch (HIP events around the phases of real batched steps) and
the fastest kept.  Results are cached in a JSON file keyed by the workload
class (sectors, field of view, density bucket, agents-per-env bucket,
clustered or not), so a class is tuned once.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import flockenv as fe

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "flockenv_tune.json")
LANES = (1, 4, 16, 64)


def workload_key(params_list, clustered=False):
    """Class of a batch: sectors, view, log2 density bucket, log2 mean agents bucket."""
    n = sum(p.n_agents for p in params_list)
    area = sum(p.box * p.box for p in params_list)
    dens = n / area if area else 0.0
    p0 = params_list[0]
    dbin = int(round(math.log2(max(dens * p0.radius ** 2, 1e-6)) * 2))
    nbin = int(round(math.log2(max(n / max(len(params_list), 1), 1))))
    full = p0.fov == 0.0 or p0.fov >= 2 * math.pi - 1e-6
    view = "full" if full else f"fov{round(math.degrees(p0.fov))}"
    return f"v{p0.obs_dim}_{view}_d{dbin}_n{nbin}_{'clustered' if clustered else 'uniform'}"


def time_sweep_lanes(batch, lanes=LANES, steps=5, warmup=2):
    """Median step time (ms, all four phases) of `batch` for each lanes value.

    The batch's envs advance by (warmup + steps) * len(lanes) steps; the
    batch is left at its automatic lane choice.
    """
    dev = batch.envs[0].workspace.device
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    act = (torch.rand(batch.n, 2, device=dev, generator=g) * 2 - 1) * torch.tensor(
        [0.2, 0.1], device=dev)
    obs = torch.empty(batch.n, batch.d, device=dev)
    rew = torch.empty(batch.n, device=dev)
    ms = {}
    for ln in lanes:
        batch.set_sweep_lanes(ln)
        for _ in range(warmup):
            batch.step(act, obs, rew)
        times = sorted(sum(batch.step_timed(act, obs, rew)) for _ in range(steps))
        ms[ln] = times[len(times) // 2]
    batch.set_sweep_lanes(0)
    return ms


def _time_config(params_list, states, reach, lanes, steps, device):
    envs = []
    for p, st in zip(params_list, states):
        q = fe.Params(**{**p.__dict__, "cell_reach": reach})
        e = fe.Env(q, device=device)
        e.set_state(*[torch.as_tensor(a).to(device) for a in st])
        e.reset()
        envs.append(e)
    b = fe.Batch(envs)
    return time_sweep_lanes(b, lanes, steps=steps)


def tune(params_list, states, clustered=False, cache=DEFAULT_CACHE, steps=5, device="cuda",
         reaches=(1, 2), lanes=LANES, force=False):
    """Best (cell reach, sweep lanes) for this batch class, timed on the batch itself.

    Returns (reach, lanes, {"r<reach>_l<lanes>": median ms per step}).  Cached
    by workload_key.
    """
    key = workload_key(params_list, clustered)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
    if not force and key in table:
        t = table[key]
        return t["reach"], t["lanes"], t["ms"]
    ms = {}
    for r in reaches:
        for ln, v in _time_config(params_list, states, r, lanes, steps, device).items():
            ms[f"r{r}_l{ln}"] = v
    best = min(ms, key=ms.get)
    reach, ln = (int(x[1:]) for x in best.split("_"))
    table[key] = {"reach": reach, "lanes": ln, "ms": ms}
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return reach, ln, ms
