"""GPU graph interaction (opinion dynamics over CSR edges) against the oracle.

One lane per node applies the edges one by one in the order the model
states, in FP64, so its FP32 output is bitwise the oracle's rounded result.
Lane groups compose chunks of a row as affine maps: the same map up to FP64
rounding, so the FP32 output is within one FP32 ulp of the oracle's.  The
threshold decision is taken in FP32 on both sides (same inputs, same
decision).  Multi-step runs are teacher-forced: each step's oracle reads the
GPU's FP32 opinions of the step before.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import workloads
from oracle import graph

pytestmark = pytest.mark.gpu
flock = pytest.importorskip("paper_2207_03945_amd")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def within_one_ulp(got, want64):
    want = want64.astype(np.float32)
    gi = got.view(np.int32).astype(np.int64)
    wi = want.view(np.int32).astype(np.int64)
    return np.abs(gi - wi) <= 1


def run_case(rp, col, w, op, thr, s, lanes, steps=1, sample=None, seed=0):
    rp_d, col_d, w_d = dev(rp.astype(np.int64)), dev(col.astype(np.int32)), dev(w.astype(np.float32))
    a, b = dev(op.astype(np.float32)), torch.empty(op.shape[0], device="cuda")
    g = np.random.default_rng(seed)
    cur = op.astype(np.float32)
    for t in range(steps):
        flock.opinion_step(rp_d, col_d, w_d, a, b, thr, s, lanes=lanes)
        got = b.cpu().numpy()
        nodes = None if sample is None else np.sort(g.choice(op.shape[0], sample, replace=False))
        want = graph.opinion_step(rp, col, w, cur, thr, s, nodes=nodes)
        rows = slice(None) if nodes is None else nodes
        if lanes == 1:
            assert np.array_equal(got[rows], want.astype(np.float32)), f"step {t}"
        else:
            ok = within_one_ulp(got[rows], want)
            assert ok.all(), f"step {t}: {np.count_nonzero(~ok)} nodes off by more than 1 ulp"
        cur = got
        a, b = b, a
    return cur


@pytest.mark.parametrize("lanes", [1, 4, 16, 64, 0])
def test_small_social_graph_every_node(lanes):
    rp, col, w = workloads.social_graph(3000, seed=1)
    op = workloads.opinions(3000, seed=1)
    run_case(rp, col, w, op, 0.3, 0.5, lanes, steps=3)


@pytest.mark.parametrize("lanes", [1, 4, 16])   # 16: the setting bench.py times
def test_million_node_graph_sampled(lanes):
    """1,000,000 nodes, ~13.8M directed edges, power-law degrees up to ~2,000."""
    rp, col, w = workloads.social_graph(1_000_000, seed=0)
    op = workloads.opinions(1_000_000, seed=0)
    run_case(rp, col, w, op, 0.3, 0.5, lanes, steps=2, sample=4000, seed=lanes)


def test_edge_cases():
    # empty rows, self edges, out-of-range columns (skipped), repeated edges, a hub
    n = 70
    edges = [(0, 0), (0, 1), (0, 1), (2, 200), (2, -5), (2, 3)] + [(5, j) for j in range(6, 70)]
    order = sorted(range(len(edges)), key=lambda k: (edges[k][0], k))
    rp = np.zeros(n + 1, np.int64)
    for me, _ in edges:
        rp[me + 1] += 1
    rp = np.cumsum(rp)
    col = np.array([edges[k][1] for k in order], np.int32)
    w = np.linspace(0.1, 1.0, len(edges)).astype(np.float32)
    op = np.random.default_rng(3).random(n).astype(np.float32)
    # the oracle skips nothing, so drop the invalid edges for its side
    valid = (col >= 0) & (col < n)
    rp_v = np.concatenate([[0], np.cumsum([valid[rp[i]:rp[i + 1]].sum() for i in range(n)])])
    for lanes in (1, 4, 16, 64):
        a, b = dev(op), torch.empty(n, device="cuda")
        flock.opinion_step(dev(rp), dev(col), dev(w), a, b, 1.0, 0.7, lanes=lanes)
        want = graph.opinion_step(rp_v, col[valid], w[valid], op, 1.0, 0.7)
        got = b.cpu().numpy()
        if lanes == 1:
            assert np.array_equal(got, want.astype(np.float32))
        else:
            assert within_one_ulp(got, want).all(), lanes


def test_empty_graph_and_zero_nodes():
    op = workloads.opinions(100, seed=4)
    rp = np.zeros(101, np.int64)
    a, b = dev(op), torch.empty(100, device="cuda")
    flock.opinion_step(dev(rp), torch.empty(0, dtype=torch.int32, device="cuda"),
                       torch.empty(0, device="cuda"), a, b, 0.3, 0.5)
    assert np.array_equal(b.cpu().numpy(), op)
    z = torch.empty(0, device="cuda")
    flock.opinion_step(torch.zeros(1, dtype=torch.int64, device="cuda"),
                       torch.empty(0, dtype=torch.int32, device="cuda"), z, z, torch.empty(0, device="cuda"),
                       0.3, 0.5)
