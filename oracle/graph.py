"""Graph interaction on the oracle side: the opinion-dynamics model (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 2.1 of arXiv:2207.03945 names interactions over the edges of a graph as
one of the engine's two base interaction patterns and illustrates it with an
opinion-dynamics model made of two interactions:

* a graph interaction over each edge (me, you) with weight w_e: when the two
  current opinions differ by less than a threshold, me's new opinion moves
  toward you's current opinion by strength * w_e,
      new_me <- (1 - strength w_e) new_me + strength w_e op_you;
* a self interaction that makes every new opinion the current one.

Readings (the text gives no more): a step is the graph interaction over all
nodes at once (every test reads the current opinions of the step's start),
then the self interaction; the new opinion starts from the current one; a
node applies its incoming edges one after another in their CSR order, so
the result is the composition of the per-edge updates in that order; edges
are directed as stored (an undirected friendship is stored both ways); the
threshold test is strict and is taken on FP32 opinions in FP32 (it decides
a branch, so both sides decide it in the same precision); the update
arithmetic is FP64 on the FP32 inputs, rounded once to FP32 at the end.
"""
from __future__ import annotations

import numpy as np


def opinion_step(row_ptr, col, weight, opinion, threshold, strength, nodes=None):
    """New opinions of `nodes` (all if None) after one step, FP64 (not yet rounded).

    ``row_ptr`` [n + 1], ``col`` [E] (the `you` of each edge), ``weight`` [E]
    and ``opinion`` [n] (FP32) describe the graph in CSR form: the incoming
    edges of node i are row_ptr[i] .. row_ptr[i + 1] - 1.
    """
    row_ptr = np.asarray(row_ptr, np.int64)
    col = np.asarray(col, np.int64)
    w32 = np.asarray(weight, np.float32)
    op32 = np.asarray(opinion, np.float32)
    thr32 = np.float32(threshold)
    strength64 = float(np.float32(strength))
    idx = np.arange(op32.shape[0]) if nodes is None else np.asarray(nodes)
    out = np.empty(idx.shape[0], np.float64)
    for r, i in enumerate(idx):
        me = op32[i]
        new = float(me)
        for e in range(row_ptr[i], row_ptr[i + 1]):
            you = op32[col[e]]
            d = np.abs(np.float32(me - you))          # FP32 decision
            if d < thr32:
                w = strength64 * float(w32[e])
                new = (1.0 - w) * new + w * float(you)
        out[r] = new
    return out
