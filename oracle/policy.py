"""Double-precision policy network (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 5 of arXiv:2207.03945 gives the actor as a network with two hidden
layers of 64 units; Sec. 4.3 states that one policy is shared by all agents,
each agent being an independent learner, so the batch axis is the agent axis.
Readings taken here (the paper gives no more): tanh activations, inputs are
the agent's v-sector view, and the action is the deterministic mean of the
policy, squashed by tanh and scaled to the action ranges of Sec. 4.1
(turn in [-max_turn, max_turn], dspeed in [-max_dspeed, max_dspeed]).
"""
from __future__ import annotations

import numpy as np


def xavier_limits(dims):
    """Glorot-uniform bound sqrt(6 / (fan_in + fan_out)) for each layer."""
    return [float(np.sqrt(6.0 / (dims[i] + dims[i + 1]))) for i in range(len(dims) - 1)]


def policy_forward(obs, weights, biases, max_turn=0.2, max_dspeed=0.1):
    """obs [n, d0] -> actions [n, 2] in float64.

    ``weights[l]`` has shape (fan_in, fan_out) and ``biases[l]`` (fan_out,).
    Hidden layers use tanh; the output layer's two pre-activations are squashed
    by tanh and scaled by (max_turn, max_dspeed).
    """
    h = np.asarray(obs, dtype=np.float64)
    n_layers = len(weights)
    for layer in range(n_layers):
        w = np.asarray(weights[layer], dtype=np.float64)
        b = np.asarray(biases[layer], dtype=np.float64)
        z = h @ w + b
        h = np.tanh(z)
    scale = np.array([max_turn, max_dspeed], dtype=np.float64)
    return h * scale
