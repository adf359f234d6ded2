"""Pins for the graph-interaction oracle (``oracle/graph.py``), CPU only.

Pinned to hand-derived cases and properties, not to itself: a two-node
exchange (closed form, and the conserved sum of a symmetric pair), the
strict threshold, the last-accepted-edge-wins limit of full-strength
updates (which fixes the edge order), the product expansion of a star's
sequential updates, consensus as a fixed point, and reading only current
opinions (a chain's far end is unaffected after one step).  A swapped
me/you, a non-strict test, a reversed edge order, reading new opinions of
other nodes or a dropped (1 - w) factor fails at least one of them.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import graph


def csr(n, edges, weights):
    """CSR of incoming edges from (me, you) pairs, keeping the given order per node."""
    order = sorted(range(len(edges)), key=lambda k: (edges[k][0], k))
    row_ptr = np.zeros(n + 1, np.int64)
    for me, _ in edges:
        row_ptr[me + 1] += 1
    row_ptr = np.cumsum(row_ptr)
    col = np.array([edges[k][1] for k in order], np.int64)
    w = np.array([weights[k] for k in order], np.float32)
    return row_ptr, col, w


def test_two_nodes_exchange_and_conserved_sum():
    rp, col, w = csr(2, [(0, 1), (1, 0)], [0.5, 0.5])
    op = np.array([0.2, 0.6], np.float32)
    new = graph.opinion_step(rp, col, w, op, threshold=0.5, strength=0.5)
    a, b = float(op[0]), float(op[1])
    np.testing.assert_allclose(new, [0.75 * a + 0.25 * b, 0.75 * b + 0.25 * a], rtol=1e-15)
    assert abs(new.sum() - (a + b)) < 1e-15


def test_threshold_is_strict_and_decided_in_fp32():
    op = np.array([0.25, 0.75], np.float32)     # exact difference 0.5
    rp, col, w = csr(2, [(0, 1)], [1.0])
    same = graph.opinion_step(rp, col, w, op, threshold=0.5, strength=0.5)
    assert same[0] == np.float32(0.25)
    above = np.nextafter(np.float32(0.5), np.float32(1))
    moved = graph.opinion_step(rp, col, w, op, threshold=above, strength=0.5)
    assert moved[0] == 0.5
    # a difference that rounds to the threshold in FP32 counts as equal (not below)
    x = np.float32(0.1)
    y = np.float32(0.1) + np.float32(0.3)
    d32 = np.abs(np.float32(x - y))
    op = np.array([x, y], np.float32)
    out = graph.opinion_step(rp, col, w, op, threshold=d32, strength=0.5)
    assert out[0] == float(x)


def test_full_strength_last_accepted_edge_wins():
    # node 0 hears 1, 2, 3 in that order; 2 is beyond the threshold
    rp, col, w = csr(4, [(0, 1), (0, 2), (0, 3)], [1.0, 1.0, 1.0])
    op = np.array([0.5, 0.45, 0.95, 0.55], np.float32)
    out = graph.opinion_step(rp, col, w, op, threshold=0.2, strength=1.0)
    assert out[0] == float(op[3])
    rp, col, w = csr(4, [(0, 3), (0, 2), (0, 1)], [1.0, 1.0, 1.0])
    out = graph.opinion_step(rp, col, w, op, threshold=0.2, strength=1.0)
    assert out[0] == float(op[1])


def test_star_product_expansion():
    g = np.random.default_rng(0)
    k = 12
    y = g.random(k).astype(np.float32) * 0.2 + 0.4
    ws = g.random(k).astype(np.float32)
    x = np.float32(0.5)
    edges = [(0, j + 1) for j in range(k)]
    rp, col, w = csr(k + 1, edges, ws)
    op = np.concatenate([[x], y]).astype(np.float32)
    s = float(np.float32(0.3))   # the model's FP32 parameter
    out = graph.opinion_step(rp, col, w, op, threshold=1.0, strength=s)[0]
    a = s * ws.astype(np.float64)
    want = np.prod(1 - a) * float(x) + sum(a[i] * float(y[i]) * np.prod(1 - a[i + 1:])
                                           for i in range(k))
    assert abs(out - want) < 1e-14


def test_consensus_fixed_point_and_zero_threshold():
    g = np.random.default_rng(1)
    n, e = 50, 400
    edges = [(int(a), int(b)) for a, b in g.integers(0, n, size=(e, 2))]
    rp, col, w = csr(n, edges, g.random(e))
    op = np.full(n, 0.3, np.float32)
    out = graph.opinion_step(rp, col, w, op, threshold=0.1, strength=0.7)
    assert (out == float(np.float32(0.3))).all()
    op = g.random(n).astype(np.float32)
    out = graph.opinion_step(rp, col, w, op, threshold=0.0, strength=0.7)
    assert (out == op.astype(np.float64)).all()


def test_reads_current_opinions_only():
    """A chain 0 <- 1 <- 2: after one step node 0 moved toward 1's old opinion only."""
    rp, col, w = csr(3, [(0, 1), (1, 2)], [1.0, 1.0])
    op = np.array([0.0, 0.2, 0.4], np.float32)
    out = graph.opinion_step(rp, col, w, op, threshold=1.0, strength=0.5)
    assert out[0] == 0.5 * float(op[1])
    assert out[1] == 0.5 * float(op[1]) + 0.5 * float(op[2])
    assert out[2] == float(op[2])


@pytest.mark.parametrize("nodes", [[0], [3, 1], None])
def test_node_subset_equals_full(nodes):
    g = np.random.default_rng(2)
    n, e = 8, 30
    edges = [(int(a), int(b)) for a, b in g.integers(0, n, size=(e, 2))]
    rp, col, w = csr(n, edges, g.random(e))
    op = g.random(n).astype(np.float32)
    full = graph.opinion_step(rp, col, w, op, 0.4, 0.5)
    part = graph.opinion_step(rp, col, w, op, 0.4, 0.5, nodes=nodes)
    want = full if nodes is None else full[nodes]
    assert np.array_equal(part, want)
