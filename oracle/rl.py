"""Experience collection on the oracle side: sampling, critic, advantages (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 4.3 and Fig. 5 of arXiv:2207.03945: every agent is an independent
learner sharing one PPO policy; each update of the simulation answers the
actions sampled from the policy, and the new views and rewards go to the
learner's experience buffer.  Sec. 5: t = 128 simulation updates per
training step, n x t trajectories, actor and critic networks of two hidden
layers of 64 units.

Readings (the paper names PPO but gives no more):
  * sampling: a diagonal Gaussian round the actor's mean action, one log
    standard deviation per action dimension; the standard-normal draws are
    an input (``eps``), so both sides see the same numbers; the log density
    of the sampled action is the Gaussian's, summed over the two dimensions;
  * critic: the actor's layer shapes with tanh hidden units and one linear
    output;
  * advantages: PPO's truncated generalised advantage estimator over the
    t-step segment, bootstrapped with the critic's value of the state after
    the last step (the flock has no terminal states inside a segment):
        delta_t = r_t + gamma V(s_{t+1}) - V(s_t)
        A_t     = delta_t + gamma lambda A_{t+1},   A_T = 0
    and the value targets R_t = A_t + V(s_t).
"""
from __future__ import annotations

import math

import numpy as np

LOG_2PI = math.log(2.0 * math.pi)


def gaussian_sample(mean, log_std, eps):
    """a = mean + exp(log_std) * eps; returns (a, log density of a), FP64.

    ``mean`` and ``eps`` are [n, k]; ``log_std`` is [k].
    """
    mean = np.asarray(mean, np.float64)
    eps = np.asarray(eps, np.float64)
    log_std = np.asarray(log_std, np.float64)
    a = mean + np.exp(log_std) * eps
    z = (a - mean) / np.exp(log_std)
    logp = np.sum(-0.5 * z * z - log_std - 0.5 * LOG_2PI, axis=-1)
    return a, logp


def value_forward(obs, weights, biases):
    """Critic: obs [n, d] -> V [n]; tanh hidden layers, linear output."""
    h = np.asarray(obs, np.float64)
    for layer, (w, b) in enumerate(zip(weights, biases)):
        z = h @ np.asarray(w, np.float64) + np.asarray(b, np.float64)
        h = np.tanh(z) if layer < len(weights) - 1 else z
    return h[:, 0]


def gae(rewards, values, gamma, lam):
    """Truncated advantage estimator: rewards [T, n], values [T+1, n] -> (A, R), FP64."""
    r = np.asarray(rewards, np.float64)
    v = np.asarray(values, np.float64)
    T = r.shape[0]
    assert v.shape[0] == T + 1
    adv = np.zeros_like(r)
    nxt = np.zeros(r.shape[1:])
    for t in range(T - 1, -1, -1):
        delta = r[t] + gamma * v[t + 1] - v[t]
        nxt = delta + gamma * lam * nxt
        adv[t] = nxt
    return adv, adv + v[:T]
