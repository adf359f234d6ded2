"""Autotuner for the batched step's cell grid.

The tunable is the cell reach r of each env: cells at least R/r wide and a
(2r + 1)^2 block of cells per agent.  r = 1 tests fewer cells with more
candidates each; r = 2 cuts candidates by about a third (25 R^2/4 vs 9 R^2
of area) at the price of more, shorter runs.  Which wins depends on the
local density and on how the runs fill the wavefronts, so it is measured:
each candidate reach is timed on the caller's own batch (HIP events around
the four phases of a real batched step) and the fastest is kept.

Results are cached in a JSON file keyed by the workload class (sectors,
density bucket, agents-per-env bucket, clustered or not), so a class is
tuned once.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import flockenv as fe

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "flockenv_tune.json")


def workload_key(params_list, clustered=False):
    """Class of a batch: sectors, log2 density bucket, log2 mean agents bucket."""
    n = sum(p.n_agents for p in params_list)
    area = sum(p.box * p.box for p in params_list)
    dens = n / area if area else 0.0
    v = params_list[0].sectors
    dbin = int(round(math.log2(max(dens * params_list[0].radius ** 2, 1e-6)) * 2))
    nbin = int(round(math.log2(max(n / max(len(params_list), 1), 1))))
    return f"v{v}_d{dbin}_n{nbin}_{'clustered' if clustered else 'uniform'}"


def _time_batch(params_list, states, reach, steps, device):
    envs = []
    for p, st in zip(params_list, states):
        q = fe.Params(**{**p.__dict__, "cell_reach": reach})
        e = fe.Env(q, device=device)
        e.set_state(*[torch.as_tensor(a).to(device) for a in st])
        e.reset()
        envs.append(e)
    b = fe.Batch(envs)
    g = torch.Generator(device=device)
    g.manual_seed(0)
    act = (torch.rand(b.n, 2, device=device, generator=g) * 2 - 1) * torch.tensor(
        [0.2, 0.1], device=device)
    obs = torch.empty(b.n, b.v, device=device)
    rew = torch.empty(b.n, device=device)
    for _ in range(3):
        b.step(act, obs, rew)
    times = [sum(b.step_timed(act, obs, rew)) for _ in range(steps)]
    times.sort()
    return times[len(times) // 2]


def tune_reach(params_list, states, clustered=False, cache=DEFAULT_CACHE, steps=7,
               device="cuda", reaches=(1, 2), force=False):
    """Best cell reach for this batch class (timed on the batch itself).

    Returns (reach, {reach: median ms per step}).  Cached by workload_key.
    """
    key = workload_key(params_list, clustered)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
    if not force and key in table:
        return table[key]["reach"], {int(k): v for k, v in table[key]["ms"].items()}
    ms = {r: _time_batch(params_list, states, r, steps, device) for r in reaches}
    best = min(ms, key=ms.get)
    table[key] = {"reach": best, "ms": {str(k): v for k, v in ms.items()}}
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best, ms
