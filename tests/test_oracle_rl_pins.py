"""Pins for the experience-collection oracle (``oracle/rl.py``), CPU only.

Each function is pinned to something other than itself: the advantage
estimator to its closed forms (lambda = 1 gives the discounted return minus
the value, lambda = 0 the one-step error, a constant reward a geometric sum)
computed here by direct sums rather than the recurrence; the Gaussian
sample's log density to scipy's normal density; the critic to its limiting
forms.  A dropped bootstrap term, a swapped gamma/lambda, an off-by-one in
the time index or a tanh on the critic's output fails at least one of them.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
from scipy import stats

from oracle import rl

import workloads


def _rand(T, n, seed):
    g = np.random.default_rng(seed)
    return g.normal(size=(T, n)), g.normal(size=(T + 1, n))


@pytest.mark.parametrize("gamma", [0.0, 0.5, 0.99, 1.0])
def test_gae_lambda_one_is_discounted_return_minus_value(gamma):
    T, n = 9, 5
    r, v = _rand(T, n, 1)
    adv, ret = rl.gae(r, v, gamma, 1.0)
    for t in range(T):
        g = sum(gamma ** k * r[t + k] for k in range(T - t)) + gamma ** (T - t) * v[T]
        np.testing.assert_allclose(adv[t], g - v[t], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(ret[t], g, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("gamma", [0.0, 0.9, 1.0])
def test_gae_lambda_zero_is_one_step_error(gamma):
    T, n = 7, 4
    r, v = _rand(T, n, 2)
    adv, ret = rl.gae(r, v, gamma, 0.0)
    np.testing.assert_allclose(adv, r + gamma * v[1:] - v[:-1], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(ret, r + gamma * v[1:], rtol=1e-13, atol=1e-13)


def test_gae_constant_reward_geometric_sum():
    T, n, c, gamma, lam = 128, 3, 0.1, 0.99, 0.95
    r = np.full((T, n), c)
    v = np.zeros((T + 1, n))
    adv, _ = rl.gae(r, v, gamma, lam)
    q = gamma * lam
    for t in (0, 1, 64, 127):
        np.testing.assert_allclose(adv[t], c * (1 - q ** (T - t)) / (1 - q), rtol=1e-12)


def test_gae_general_against_explicit_sum():
    """A_t = sum_k (gamma lambda)^k delta_{t+k}, written out."""
    T, n, gamma, lam = 12, 6, 0.97, 0.9
    r, v = _rand(T, n, 3)
    adv, _ = rl.gae(r, v, gamma, lam)
    delta = r + gamma * v[1:] - v[:-1]
    for t in range(T):
        want = sum((gamma * lam) ** k * delta[t + k] for k in range(T - t))
        np.testing.assert_allclose(adv[t], want, rtol=1e-12, atol=1e-12)


def test_gae_agents_independent():
    T, n = 5, 8
    r, v = _rand(T, n, 4)
    full, _ = rl.gae(r, v, 0.9, 0.8)
    perm = np.random.default_rng(5).permutation(n)
    part, _ = rl.gae(r[:, perm], v[:, perm], 0.9, 0.8)
    np.testing.assert_array_equal(part, full[:, perm])


def test_gaussian_logp_matches_scipy():
    g = np.random.default_rng(6)
    mean = g.normal(size=(50, 2)) * 0.1
    eps = g.normal(size=(50, 2))
    log_std = np.array([-1.3, -2.0])
    a, logp = rl.gaussian_sample(mean, log_std, eps)
    np.testing.assert_allclose(a, mean + np.exp(log_std) * eps, rtol=1e-15)
    want = stats.norm.logpdf(a, loc=mean, scale=np.exp(log_std)).sum(axis=1)
    np.testing.assert_allclose(logp, want, rtol=1e-12, atol=1e-12)
    # eps = 0: the density peak
    _, lp0 = rl.gaussian_sample(mean, log_std, np.zeros_like(eps))
    np.testing.assert_allclose(lp0, -log_std.sum() - math.log(2 * math.pi), rtol=1e-14)


def test_value_forward_limits():
    dims = [129, 64, 64, 1]
    ws, bs = workloads.xavier_weights(dims, seed=7)
    ws = [w.astype(np.float64) for w in ws]
    bs = [b.astype(np.float64) for b in bs]
    obs = np.random.default_rng(8).random((20, 129))
    # zero weights: the output bias
    zw = [np.zeros_like(w) for w in ws]
    b3 = np.array([0.75])
    np.testing.assert_array_equal(rl.value_forward(obs, zw, [bs[0], bs[1], b3]), np.full(20, 0.75))
    # linear output: scaling the last layer scales V (no squashing)
    v1 = rl.value_forward(obs, ws, bs)
    v3 = rl.value_forward(obs, ws[:2] + [ws[2] * 3.0], bs)
    np.testing.assert_allclose(v3, 3.0 * v1, rtol=1e-13)
    # large last-layer weights are not clipped to [-1, 1]
    big = rl.value_forward(obs, ws[:2] + [ws[2] * 100.0], bs)
    assert np.abs(big).max() > 1.0
    # hidden layers are tanh: odd symmetry with zero biases
    np.testing.assert_allclose(rl.value_forward(-obs, ws, bs), -v1, rtol=1e-13, atol=1e-15)
