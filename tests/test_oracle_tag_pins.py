"""Pins for the tag-environment oracle (Sec. 4.2), CPU only.

Pinned to the flock oracle's special case (no chasers: the runner channel is
the flock view and the reward the flock's proximity term), hand-derived
two-agent cases for every type pair, the balance of touches between the two
types, permutation within a type, and the move's direct-speed closed forms.
A swapped channel, a touch counted within a type, a missing penalty or a
speed read as an acceleration fails at least one of them.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import workloads

R = 8.0


def sense2(pos_a, pos_b, th_a, n_chasers, v=8, box=64.0):
    x = np.array([pos_a[0], pos_b[0]], np.float32)
    y = np.array([pos_a[1], pos_b[1]], np.float32)
    th = np.array([th_a, 0.0], np.float32)
    return oracle.oracle_sense_tag(x, y, th, box, n_chasers, radius=R, touch=0.5, sectors=v)


def test_no_chasers_reduces_to_flock():
    st = workloads.uniform_state(400, 64.0, seed=3)
    tag = oracle.oracle_sense_tag(st[0], st[1], st[2], 64.0, 0, radius=R, touch=0.5, sectors=16)
    flk = oracle.oracle_sense(st[0], st[1], st[2], 64.0, radius=R, collide=0.5, sectors=16,
                              r_nb=0.1, r_col=0.0)
    np.testing.assert_array_equal(tag.obs[:, :16], flk.obs)
    assert not tag.obs[:, 16:].any()
    np.testing.assert_array_equal(tag.n_nb, flk.n_nb)
    assert not tag.n_col.any()
    np.testing.assert_allclose(tag.reward, flk.reward, rtol=1e-15)


def test_chaser_touches_runner():
    # agent 0 is the chaser; agent 1 a runner 0.3 straight ahead of it (heading 0)
    s = sense2((10.0, 10.0), (10.3, 10.0), 0.0, n_chasers=1)
    assert list(s.n_col) == [1, 1]
    assert s.reward[0] == 1.0            # chaser: +1 per runner touched
    assert s.reward[1] == -1.0           # runner: no runner near, one chaser touching
    d = float(np.float32(10.3)) - 10.0
    assert s.obs[0, 0] == pytest.approx(1 - d / R)       # chaser sees a runner ahead: channel 0
    assert not s.obs[0, 8:].any()
    # the runner's heading is 0 too; the chaser lies behind it: bearing pi -> sector 4 of 8
    assert s.obs[1, 8 + 4] == pytest.approx(1 - d / R)   # runner sees a chaser: channel 1
    assert not s.obs[1, :8].any()


def test_runner_pair_and_chaser_pair():
    s = sense2((10.0, 10.0), (10.3, 10.0), 0.0, n_chasers=0)   # two runners, touching
    assert list(s.n_col) == [0, 0] and list(s.n_nb) == [1, 1]
    np.testing.assert_allclose(s.reward, [0.1, 0.1], rtol=1e-15)
    s = sense2((10.0, 10.0), (10.3, 10.0), 0.0, n_chasers=2)   # two chasers, touching
    assert list(s.n_col) == [0, 0] and list(s.n_nb) == [0, 0]
    assert list(s.reward) == [0.0, 0.0]
    assert s.obs[0, 8] > 0 and not s.obs[0, :8].any()


def test_runner_near_other_runner_and_chaser_far():
    # runner 1 at distance 5 (in range, no touch) from chaser 0; runners 1 and 2 at distance 3
    x = np.array([10.0, 15.0, 18.0], np.float32)
    y = np.array([10.0, 10.0, 10.0], np.float32)
    th = np.zeros(3, np.float32)
    s = oracle.oracle_sense_tag(x, y, th, 64.0, 1, radius=R, touch=0.5, sectors=8)
    assert list(s.n_nb) == [1, 1, 1]      # runners in range: chaser sees 1 (8 away is out)
    assert list(s.n_col) == [0, 0, 0]
    np.testing.assert_allclose(s.reward, [0.0, 0.1, 0.1], rtol=1e-15)


def test_touches_balance_between_types():
    st = workloads.blob_state(600, 100.0, seed=4, n_blobs=8)
    s = oracle.oracle_sense_tag(st[0], st[1], st[2], 100.0, 55, radius=R, touch=2.0, sectors=16)
    assert s.n_col[:55].sum() == s.n_col[55:].sum() > 0


def test_permutation_within_types():
    st = workloads.uniform_state(300, 50.0, seed=5)
    nc = 27
    perm = np.concatenate([np.random.default_rng(1).permutation(nc),
                           nc + np.random.default_rng(2).permutation(300 - nc)])
    a = oracle.oracle_sense_tag(st[0], st[1], st[2], 50.0, nc, radius=R, touch=1.0, sectors=16)
    b = oracle.oracle_sense_tag(st[0][perm], st[1][perm], st[2][perm], 50.0, nc, radius=R,
                                touch=1.0, sectors=16)
    np.testing.assert_array_equal(b.obs, a.obs[perm])
    np.testing.assert_array_equal(b.n_col, a.n_col[perm])
    np.testing.assert_array_equal(b.reward, a.reward[perm])


def test_move_uses_speed_directly():
    x = np.array([5.0, 5.0, 5.0, 63.5], np.float32)
    y = np.array([5.0, 5.0, 5.0, 1.0], np.float32)
    th = np.zeros(4, np.float32)
    s = np.full(4, 1.5, np.float32)
    act = np.array([[0.0, 1.0], [0.0, -3.0], [0.1, 7.0], [0.0, 1.0]], np.float32)
    nx, ny, nth, ns = oracle.oracle_move_tag((x, y, th, s), act, 64.0, max_turn=0.2, s_max=2.0)
    assert ns.tolist() == [1.0, 0.0, 2.0, 1.0]        # speed = clamp(a1, 0, s_max), not s + a1
    assert nx[0] == np.float32(6.0) and ny[0] == np.float32(5.0)
    assert nx[1] == np.float32(5.0)                     # speed 0: stays
    assert nth[2] == np.float32(0.1)
    c = np.float32(math.cos(float(np.float32(0.1))))
    assert nx[2] == np.float32(np.float32(5.0) + np.float32(2.0) * c)
    assert nx[3] == np.float32(0.5)                     # wraps
