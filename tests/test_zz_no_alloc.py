"""env_step_static (the step whose scratch lives in the library's static device
array) against env_step, through the C ABI: bitwise equal view, reward,
counts, state and FP64 returns on twin envs, over two calls in a row of which
the second steps a smaller env, then the rejection of a step that needs more
scratch than the array holds."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

flock = pytest.importorskip("paper_2207_03945_amd")
from paper_2207_03945_amd import flockenv  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def twins(n, seed, lanes=0):
    box = float(np.float32(4.0 * math.sqrt(n)))
    st = workloads.uniform_state(n, box, seed=seed)
    envs = []
    for _ in range(2):
        e = flock.Env(flock.Params(n_agents=n, box=box, sectors=16, flags=flock.ENV_FLAG_COUNTS))
        if lanes:
            e.set_sweep_lanes(lanes)
        e.set_state(*[dev(a) for a in st])
        e.reset()
        envs.append(e)
    return envs


def same(a, b, what):
    a, b = a.cpu(), b.cpu()
    assert a.shape == b.shape, what
    ok = torch.equal(a.view(torch.int32) if a.dtype == torch.float32 else
                     a.view(torch.int64) if a.dtype == torch.float64 else a,
                     b.view(torch.int32) if b.dtype == torch.float32 else
                     b.view(torch.int64) if b.dtype == torch.float64 else b)
    assert ok, f"{what} differs"


def step_pair(ref, sta, act, label):
    o1, r1 = ref.step(act)
    o2, r2 = sta.step_static(act)
    torch.cuda.synchronize()
    same(o1, o2, f"{label} obs")
    same(r1, r2, f"{label} reward")
    for a, b, nm in zip(ref.counts(), sta.counts(), ("n_nb", "n_col")):
        same(a, b, f"{label} {nm}")
    for a, b, nm in zip(ref.get_state(), sta.get_state(), "x y th s".split()):
        same(a, b, f"{label} {nm}")
    same(ref.returns(), sta.returns(), f"{label} returns")


@pytest.mark.parametrize("lanes", [0, 1])
def test_static_step_equals_step_then_smaller(lanes):
    assert flock.lib().env_static_scratch_bytes() == 32 << 20
    big = twins(60_000, seed=31, lanes=lanes)
    small = twins(3_000, seed=37, lanes=lanes)
    for t in range(2):
        act = dev(workloads.random_actions(60_000, seed=31, step=t))
        step_pair(*big, act, f"60k step {t}")
        act = dev(workloads.random_actions(3_000, seed=37, step=t))
        step_pair(*small, act, f"3k step {t}")


def test_static_step_rejects_oversize_before_launch():
    n = 1_200_000
    box = float(np.float32(4.0 * math.sqrt(n)))
    e = flock.Env(flock.Params(n_agents=n, box=box, sectors=16))
    act = torch.zeros(n, 2, device="cuda")
    with pytest.raises(flock.FlockError) as ei:
        e.step_static(act)
    assert ei.value.code == flockenv.ENV_ENOMEM
    assert "static array" in str(ei.value)
