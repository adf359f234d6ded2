"""Pins for the CPU oracle (no GPU).

The oracle is pinned to things other than itself: hand-derived closed forms
(tests/golden/closed_forms.txt), integer lattice enumeration, exact symmetry
and invariance properties, the expected neighbour count of a uniform Poisson
cloud, straight-line motion and clamp saturation, a correctly rounded cosine
computed with decimal arithmetic, and the limiting forms of the policy
network.  Each is chosen so that a plausible slip (wrong image, sign or index,
swapped atan2 arguments, non-strict radius test, dropped collision term,
transposed weight) fails at least one of them.
"""
from __future__ import annotations

import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.txt")


def _golden(kind):
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == kind:
                rows.append([float(p) for p in parts[1:]])
    return rows


def _lattice(a, box, heading):
    m = int(round(box / a))
    ii, jj = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    x = (ii.ravel() * a).astype(np.float32)
    y = (jj.ravel() * a).astype(np.float32)
    th = np.full(x.shape, heading, np.float32)
    return x, y, th


def _gauss_count(q2):
    r = math.isqrt(int(q2)) + 1
    return sum(1 for i in range(-r, r + 1) for j in range(-r, r + 1) if 0 < i * i + j * j < q2)


# --------------------------------------------------------------------------- lattices

@pytest.mark.parametrize("row", _golden("lattice"), ids=lambda r: f"a={r[0]}")
def test_lattice_counts_reward_obs(oracle_mod, row):
    a, box, n_nb, n_col, reward, obs_axis, obs_diag = row
    # the stored counts are the integer-lattice (Gauss circle) counts
    assert _gauss_count((8.0 / a) ** 2) == n_nb
    assert _gauss_count((0.5 / a) ** 2) == n_col
    x, y, th = _lattice(a, box, 0.1)
    n = x.shape[0]
    agents = np.array([0, 1, n // 2 + 7, n - 1], np.int32)
    r = oracle_mod.oracle_sense(x, y, th, box, sectors=8, agents=agents)
    assert (r.n_nb == n_nb).all(), r.n_nb
    assert (r.n_col == n_col).all(), r.n_col
    np.testing.assert_allclose(r.reward, reward, rtol=1e-12)
    expect = np.array([obs_diag, obs_axis] * 4)
    np.testing.assert_allclose(r.obs, np.tile(expect, (len(agents), 1)), rtol=0, atol=1e-12)


# --------------------------------------------------------------------------- two agents

@pytest.mark.parametrize("row", _golden("pair"), ids=lambda r: f"xj={r[5]},yj={r[6]}")
def test_two_agent_closed_forms(oracle_mod, row):
    box, v, xi, yi, thi, xj, yj, sector, obs, nb, col, reward = row
    v, sector = int(v), int(sector)
    x = np.array([xi, xj], np.float32)
    y = np.array([yi, yj], np.float32)
    th = np.array([thi, 0.0], np.float32)
    r = oracle_mod.oracle_sense(x, y, th, box, sectors=v, agents=[0])
    expect = np.zeros(v)
    if sector >= 0:
        expect[sector] = obs
    np.testing.assert_allclose(r.obs[0], expect, rtol=0, atol=1e-12)
    assert r.n_nb[0] == nb and r.n_col[0] == col
    np.testing.assert_allclose(r.reward[0], reward, rtol=0, atol=1e-12)


def test_pair_bearing_every_sector(oracle_mod):
    """j placed at the centre of each sector in turn is seen in that sector."""
    v, d = 16, 3.0
    for heading in (0.0, 1.3, 5.9):
        for k in range(v):
            beta = heading + (k + 0.5) * 2 * math.pi / v
            x = np.array([32.0, 32.0 + d * math.cos(beta)], np.float32)
            y = np.array([32.0, 32.0 + d * math.sin(beta)], np.float32)
            th = np.array([heading, 0.0], np.float32)
            r = oracle_mod.oracle_sense(x, y, th, 64.0, sectors=v, agents=[0])
            assert int(np.argmax(r.obs[0])) == k
            assert np.count_nonzero(r.obs[0]) == 1


# --------------------------------------------------------------------------- invariants

def _dyadic_state(n, box, seed, frac_bits=10):
    g = np.random.default_rng(seed)
    q = 2.0 ** -frac_bits
    x = (np.floor(g.random(n) * box / q) * q).astype(np.float32)
    y = (np.floor(g.random(n) * box / q) * q).astype(np.float32)
    th = (g.random(n) * 2 * math.pi).astype(np.float32)
    return x, y, th


@pytest.mark.parametrize("init", ["uniform", "blobs"])
def test_relation_symmetric(oracle_mod, init):
    n, box = 3000, 200.0
    if init == "uniform":
        x, y, th, _ = workloads.uniform_state(n, box, seed=3)
    else:
        x, y, th, _ = workloads.blob_state(n, box, seed=3, n_blobs=8, sigma=4.0)
    r = oracle_mod.oracle_sense(x, y, th, box)
    assert r.n_nb.sum() % 2 == 0 and r.n_col.sum() % 2 == 0
    assert r.n_col.sum() > 0 or init == "uniform"
    # the sum over agents of the reward equals the reward of the pair set counted twice
    np.testing.assert_allclose(r.reward.sum(), 0.1 * r.n_nb.sum() - r.n_col.sum(), rtol=1e-12)


def test_symmetric_pairwise_distance(oracle_mod):
    """For every pair inside R, the distance each side reports is the same.

    Each agent here has exactly one neighbour, so obs identifies the distance.
    """
    g = np.random.default_rng(11)
    box, pairs = 64.0, []
    xs, ys = [], []
    for k in range(12):
        cx, cy = (k % 4) * 16.0 + 1.0, (k // 4) * 21.0 + 1.0  # pairs far apart, some on seams
        d, beta = 0.3 + 7.0 * g.random(), 2 * math.pi * g.random()
        xs += [cx, (cx + d * math.cos(beta)) % box]
        ys += [cy, (cy + d * math.sin(beta)) % box]
        pairs.append((2 * k, 2 * k + 1))
    x = np.array(xs, np.float32)
    y = np.array(ys, np.float32)
    th = (g.random(len(xs)) * 6.28).astype(np.float32)
    r = oracle_mod.oracle_sense(x, y, th, box, sectors=8)
    for i, j in pairs:
        assert r.n_nb[i] == 1 and r.n_nb[j] == 1
        assert abs(r.obs[i].max() - r.obs[j].max()) < 1e-15


def test_permutation_invariance(oracle_mod):
    n, box = 1200, 120.0
    x, y, th, _ = workloads.uniform_state(n, box, seed=5)
    r = oracle_mod.oracle_sense(x, y, th, box)
    p = np.random.default_rng(0).permutation(n)
    rp = oracle_mod.oracle_sense(x[p], y[p], th[p], box)
    assert np.array_equal(rp.obs, r.obs[p])
    assert np.array_equal(rp.n_nb, r.n_nb[p]) and np.array_equal(rp.n_col, r.n_col[p])


def test_translation_invariance(oracle_mod):
    """Exact periodic translation (dyadic positions) leaves the view unchanged."""
    n, box = 1500, 64.0
    x, y, th = _dyadic_state(n, box, 7)
    r = oracle_mod.oracle_sense(x, y, th, box)
    for sx, sy in ((16.0, 0.0), (0.0, 40.5), (63.0, 33.25)):
        xt = np.mod(x.astype(np.float64) + sx, box).astype(np.float32)
        yt = np.mod(y.astype(np.float64) + sy, box).astype(np.float32)
        rt = oracle_mod.oracle_sense(xt, yt, th, box)
        assert np.array_equal(rt.n_nb, r.n_nb) and np.array_equal(rt.n_col, r.n_col)
        np.testing.assert_allclose(rt.obs, r.obs, rtol=0, atol=1e-12)


def test_quarter_turn_invariance(oracle_mod):
    """Rotating positions and headings by 90 degrees keeps every sector (v % 4 == 0).

    (x, y) -> (-y, x) is exact on dyadic positions; the heading gains pi/2
    (rounded to FP32), so pairs within 1e-5 rad of a sector edge are skipped.
    """
    n, box, v = 1500, 64.0, 8
    x, y, th = _dyadic_state(n, box, 9)
    r = oracle_mod.oracle_sense(x, y, th, box, sectors=v, eps_phi=1e-5)
    xr = np.mod(-y.astype(np.float64), box).astype(np.float32)
    yr = x.copy()
    thr = np.mod(th.astype(np.float64) + math.pi / 2, 2 * math.pi).astype(np.float32)
    rr = oracle_mod.oracle_sense(xr, yr, thr, box, sectors=v, eps_phi=1e-5)
    assert np.array_equal(rr.n_nb, r.n_nb)
    clean = np.isclose(r.dmin_strict, r.dmin_loose) | (np.isinf(r.dmin_strict) & np.isinf(r.dmin_loose))
    assert clean.mean() > 0.95
    np.testing.assert_allclose(rr.obs[clean], r.obs[clean], rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,box", [(5000, 316.0), (4000, 150.0)])
def test_mean_neighbours_poisson(oracle_mod, n, box):
    """Uniform cloud: E[n_nb] = (N-1) pi R^2 / L^2, E[n_col] = (N-1) pi r_c^2 / L^2."""
    x, y, th, _ = workloads.uniform_state(n, box, seed=1)
    r = oracle_mod.oracle_sense(x, y, th, box)
    p_nb = math.pi * 64.0 / box ** 2
    mean = (n - 1) * p_nb
    sigma = math.sqrt(2.0 * mean / n)
    assert abs(r.n_nb.mean() - mean) < 5 * sigma
    mean_c = (n - 1) * math.pi * 0.25 / box ** 2
    assert abs(r.n_col.mean() - mean_c) < 5 * math.sqrt(2.0 * mean_c / n) + 1e-9


def test_empty_view_far_apart(oracle_mod):
    x = np.array([1.0, 30.0, 1.0], np.float32)
    y = np.array([1.0, 30.0, 33.0], np.float32)
    th = np.zeros(3, np.float32)
    r = oracle_mod.oracle_sense(x, y, th, 64.0, sectors=8)
    assert (r.obs == 0).all() and (r.n_nb == 0).all() and (r.reward == 0).all()


def test_bands_collapse_and_cover(oracle_mod):
    n, box = 2000, 100.0
    x, y, th, _ = workloads.uniform_state(n, box, seed=2)
    plain = oracle_mod.oracle_sense(x, y, th, box)
    band = oracle_mod.oracle_sense(x, y, th, box, eps_d=1e-3, eps_phi=1e-3)
    assert (band.nb_lo <= plain.n_nb).all() and (plain.n_nb <= band.nb_hi).all()
    assert (band.col_lo <= plain.n_col).all() and (plain.n_col <= band.col_hi).all()
    dplain = np.where(plain.obs > 0, (1 - plain.obs) * 8.0, np.inf)
    assert (band.dmin_loose <= dplain + 1e-12).all()
    assert (dplain <= band.dmin_strict + 1e-12).all()
    zero = oracle_mod.oracle_sense(x, y, th, box, eps_d=0.0, eps_phi=0.0)
    assert np.array_equal(zero.nb_lo, zero.nb_hi)
    assert np.array_equal(zero.dmin_strict, zero.dmin_loose)


# --------------------------------------------------------------------------- move

def _run_moves(oracle_mod, state, act, steps, box=64.0):
    for _ in range(steps):
        state = oracle_mod.oracle_move(state, act, box)
    return state


def test_straight_line_motion(oracle_mod):
    n = 4
    x = np.array([0.5, 10.25, 62.5, 33.0], np.float32)
    y = np.array([3.0, 7.5, 12.0, 60.0], np.float32)
    state = (x, y, np.zeros(n, np.float32), np.ones(n, np.float32))
    act = np.zeros((n, 2), np.float32)
    out = _run_moves(oracle_mod, state, act, 37)
    np.testing.assert_array_equal(out[0], np.mod(x + 37.0, 64.0).astype(np.float32))
    np.testing.assert_array_equal(out[1], y)
    # heading pi_f: cos = -1 exactly, |sin| < half an ulp of y >= 2, so y stays
    state = (x, y, np.full(n, math.pi, np.float32), np.ones(n, np.float32))
    out = _run_moves(oracle_mod, state, act, 5)
    np.testing.assert_array_equal(out[0], np.mod(x.astype(np.float64) - 5.0, 64.0).astype(np.float32))
    np.testing.assert_array_equal(out[1], y)


def test_wrap_edges(oracle_mod):
    box = 64.0
    x = np.array([63.5, 0.25, 63.75, 0.0], np.float32)
    y = np.array([5.0, 5.0, 63.5, 5.0], np.float32)
    th = np.array([0.0, math.pi, 0.0, math.pi], np.float32)
    s = np.array([1.0, 1.0, 0.25, 0.0], np.float32)
    act = np.zeros((4, 2), np.float32)
    out = oracle_mod.oracle_move((x, y, th, s), act, box)
    np.testing.assert_array_equal(out[0], np.array([0.5, 63.25, 0.0, 0.0], np.float32))
    assert ((out[0] >= 0) & (out[0] < box)).all() and ((out[1] >= 0) & (out[1] < box)).all()


def test_speed_clamp_saturates(oracle_mod):
    n = 2
    state = (np.full(n, 10.0, np.float32), np.full(n, 10.0, np.float32),
             np.zeros(n, np.float32), np.ones(n, np.float32))
    act = np.array([[0.0, 0.1], [0.0, -0.1]], np.float32)
    seen = []
    for _ in range(15):
        state = oracle_mod.oracle_move(state, act, 64.0)
        seen.append(state[3].copy())
    seen = np.array(seen)
    assert seen[:, 0].max() == np.float32(2.0) and seen[-1, 0] == np.float32(2.0)
    assert seen[:, 1].min() == np.float32(0.0) and seen[-1, 1] == np.float32(0.0)
    assert (np.diff(seen[:, 0]) >= 0).all() and (np.diff(seen[:, 1]) <= 0).all()


def test_move_uses_new_heading_and_speed(oracle_mod):
    """dt = 1 and the position advances with the speed and heading after the action."""
    n = 3
    x = np.array([10.0, 20.0, 30.0], np.float32)
    y = np.array([10.0, 20.0, 30.0], np.float32)
    th = np.array([0.0, 0.0, math.pi], np.float32)
    s = np.ones(n, np.float32)
    act = np.array([[0.0, 0.1], [0.0, -0.1], [0.0, 0.05]], np.float32)
    out = oracle_mod.oracle_move((x, y, th, s), act, 64.0)
    new_s = s + act[:, 1]
    np.testing.assert_array_equal(out[3], new_s)
    np.testing.assert_array_equal(out[0], np.array([x[0] + new_s[0], x[1] + new_s[1],
                                                    x[2] - new_s[2]], np.float32))
    # a quarter turn from heading 0 by the clamp limit moves along (cos 0.2, sin 0.2)
    out = oracle_mod.oracle_move((x[:1], y[:1], th[:1], s[:1]), np.array([[0.2, 0.0]], np.float32), 64.0)
    assert out[2][0] == np.float32(0.2)
    assert out[1][0] > y[0] + 0.19 and out[0][0] < x[0] + 0.99


def test_action_clamp_and_nan(oracle_mod):
    n = 4
    state = (np.full(n, 10.0, np.float32), np.full(n, 10.0, np.float32),
             np.full(n, 1.0, np.float32), np.ones(n, np.float32))
    act = np.array([[5.0, 5.0], [-5.0, -5.0], [np.nan, np.nan], [0.05, 0.0]], np.float32)
    out = oracle_mod.oracle_move(state, act, 64.0)
    np.testing.assert_array_equal(out[2], np.float32(1.0) + np.array([0.2, -0.2, -0.2, 0.05], np.float32))
    np.testing.assert_array_equal(out[3], np.float32(1.0) + np.array([0.1, -0.1, -0.1, 0.0], np.float32))


def test_heading_wrap(oracle_mod):
    th = np.array([6.2, 0.1, 0.0, 6.28318], np.float32)
    act = np.array([[0.2, 0], [-0.2, 0], [-0.0, 0], [0.2, 0]], np.float32)
    n = 4
    out = oracle_mod.oracle_move((np.full(n, 9.0, np.float32), np.full(n, 9.0, np.float32), th,
                                  np.zeros(n, np.float32)), act, 64.0)
    two_pi_f = np.float32(2 * math.pi)
    assert ((out[2] >= 0) & (out[2] < two_pi_f)).all()
    np.testing.assert_array_equal(out[2][0], (th[0] + np.float32(0.2)) - two_pi_f)
    np.testing.assert_array_equal(out[2][1], (th[1] - np.float32(0.2)) + two_pi_f)


def _decimal_cos_sin(theta: float):
    getcontext().prec = 60
    t = Decimal(theta)
    c, s, term_c, term_s = Decimal(0), Decimal(0), Decimal(1), t
    for k in range(60):
        c += term_c
        s += term_s
        term_c = -term_c * t * t / ((2 * k + 1) * (2 * k + 2))
        term_s = -term_s * t * t / ((2 * k + 2) * (2 * k + 3))
    return c, s


def test_cos_sin_correctly_rounded(oracle_mod):
    """With x = y = 0, s' = 1 and a positive cosine/sine the new position is fl32(cos), fl32(sin)."""
    hs = np.array([0.3, 0.7777, 1.2, 0.05, 1.5], np.float32)
    n = hs.shape[0]
    out = oracle_mod.oracle_move((np.zeros(n, np.float32), np.zeros(n, np.float32), hs,
                                  np.ones(n, np.float32)), np.zeros((n, 2), np.float32), 64.0)
    for k in range(n):
        c, s = _decimal_cos_sin(float(hs[k]))
        assert out[0][k] == np.float32(float(c))
        assert out[1][k] == np.float32(float(s))


# --------------------------------------------------------------------------- policy

DIMS = [16, 64, 64, 2]


def test_policy_zero_and_saturation(oracle_mod):
    obs = np.random.default_rng(0).random((10, 16))
    ws = [np.zeros((DIMS[i], DIMS[i + 1])) for i in range(3)]
    bs = [np.zeros(DIMS[i + 1]) for i in range(3)]
    assert (oracle_mod.policy_forward(obs, ws, bs) == 0).all()
    ws = [np.full((DIMS[i], DIMS[i + 1]), 50.0) for i in range(3)]
    act = oracle_mod.policy_forward(obs + 0.1, ws, bs)
    np.testing.assert_allclose(act, np.tile([0.2, 0.1], (10, 1)), rtol=0, atol=1e-15)


def test_policy_odd_symmetry_and_linear_regime(oracle_mod):
    ws, bs = workloads.xavier_weights(DIMS, seed=1)
    ws = [w.astype(np.float64) for w in ws]
    bs = [b.astype(np.float64) for b in bs]
    obs = np.random.default_rng(2).random((32, 16))
    a = oracle_mod.policy_forward(obs, ws, bs)
    np.testing.assert_allclose(oracle_mod.policy_forward(-obs, ws, bs), -a, rtol=0, atol=1e-15)
    eps = 1e-4
    small = [w * eps for w in ws]
    lin = obs @ ws[0] @ ws[1] @ ws[2] * eps ** 3 * np.array([0.2, 0.1])
    got = oracle_mod.policy_forward(obs, small, bs)
    np.testing.assert_allclose(got, lin, rtol=1e-6, atol=0)
    # bias of the last layer shifts the pre-activation
    b3 = np.array([0.5, -0.25])
    zero_w = [np.zeros_like(w) for w in ws]
    got = oracle_mod.policy_forward(obs, zero_w, [bs[0], bs[1], b3])
    np.testing.assert_allclose(got, np.tile(np.tanh(b3) * [0.2, 0.1], (32, 1)), rtol=1e-15)


def test_xavier_bounds_and_variance():
    ws, bs = workloads.xavier_weights(DIMS, seed=0)
    for w, (fi, fo) in zip(ws, zip(DIMS[:-1], DIMS[1:])):
        a = math.sqrt(6.0 / (fi + fo))
        assert w.shape == (fi, fo) and np.abs(w).max() <= a
        if w.size > 1000:
            assert abs(w.var() - a * a / 3) < 0.1 * a * a / 3
    assert sum(w.size + b.size for w, b in zip(ws, bs)) == 5378


# --------------------------------------------------------------------------- field of view

FOV250 = math.radians(250.0)


@pytest.mark.parametrize("bearing_deg,sector", [(180.0, -1), (100.0, 7), (-124.0, 0), (-126.0, -1),
                                                (10.0, 4), (-10.0, 3), (124.0, 7), (126.0, -1)])
def test_fov_two_agent(oracle_mod, bearing_deg, sector):
    """250-degree view, 8 sectors of 31.25 degrees from the right edge (-125 deg)."""
    d, heading = 3.0, 0.7
    b = heading + math.radians(bearing_deg)
    x = np.array([32.0, 32.0 + d * math.cos(b)], np.float32)
    y = np.array([32.0, 32.0 + d * math.sin(b)], np.float32)
    th = np.array([heading, 0.0], np.float32)
    r = oracle_mod.oracle_sense(x, y, th, 64.0, sectors=8, agents=[0], fov=FOV250)
    expect = np.zeros(8)
    if sector >= 0:
        expect[sector] = 1.0 - d / 8.0
    np.testing.assert_allclose(r.obs[0], expect, rtol=0, atol=1e-6)
    # the reward does not depend on the view (Eq. (1) sums over d < d_v)
    assert r.n_nb[0] == 1 and abs(r.reward[0] - 0.1) < 1e-12


def test_fov_coincident_is_straight_ahead(oracle_mod):
    x = np.array([5.0, 5.0], np.float32)
    th = np.array([2.0, 0.0], np.float32)
    r = oracle_mod.oracle_sense(x, x.copy(), th, 64.0, sectors=8, agents=[0], fov=FOV250)
    assert r.obs[0][4] == 1.0 and np.count_nonzero(r.obs[0]) == 1


def test_half_view_equals_rotated_full_view(oracle_mod):
    """A pi-wide view with 8 sectors is the first 8 of 16 full-view sectors
    of the same agent turned by -pi/2 (the view's right edge)."""
    n, box = 1500, 100.0
    x, y, th, _ = workloads.uniform_state(n, box, seed=12)
    half = oracle_mod.oracle_sense(x, y, th, box, sectors=8, fov=math.pi, eps_phi=1e-5)
    th2 = np.mod(th.astype(np.float64) - math.pi / 2, 2 * math.pi).astype(np.float32)
    full = oracle_mod.oracle_sense(x, y, th2, box, sectors=16, eps_phi=1e-5)
    a, b = half.dmin_strict, full.dmin_strict[:, :8]
    clean = (a == half.dmin_loose) & (b == full.dmin_loose[:, :8])
    assert clean.mean() > 0.97
    np.testing.assert_allclose(half.obs[clean], full.obs[:, :8][clean], rtol=0, atol=1e-12)
    assert np.array_equal(half.n_nb, full.n_nb)


def test_fov_only_hides_never_adds(oracle_mod):
    n, box = 2000, 120.0
    x, y, th, _ = workloads.uniform_state(n, box, seed=4)
    full = oracle_mod.oracle_sense(x, y, th, box, sectors=16)
    lim = oracle_mod.oracle_sense(x, y, th, box, sectors=16, fov=FOV250)
    assert np.array_equal(full.reward, lim.reward)
    # the nearest visible agent can never be nearer than the nearest agent
    assert (lim.obs.max(axis=1) <= full.obs.max(axis=1) + 1e-15).all()
    assert (lim.obs > 0).sum() < (full.obs > 0).sum()


def test_observation_appends_speed(oracle_mod):
    x, y, th, s = workloads.uniform_state(50, 40.0, seed=1)
    s = (np.arange(50) * 0.03).astype(np.float32)
    r = oracle_mod.oracle_sense(x, y, th, 40.0, sectors=8, agents=[3, 7])
    o = oracle_mod.observation(r, s)
    assert o.shape == (2, 9) and o[0, 8] == np.float32(0.09) and o[1, 8] == np.float32(0.21)


# --------------------------------------------------------------------------- band widths
#
# The ambiguity bands decide how far the GPU parity tests may stray from the
# plain definition, so their WIDTH is pinned here, not only their containment:
# a pair 0.5e-5 from a radius or a sector edge must be ambiguous, a pair 2e-5
# away must not be.  The offsets are measured in the test from the FP32
# coordinates themselves (exact differences in double, math.hypot and
# math.atan2), so a band applied to d^2 instead of d, or a sector band scaled
# by the wrong arc, fails one of these cases.

EPS = 1e-5


def _pair_at(d, bearing, heading=0.0, x0=9.0, y0=9.0):
    x = np.array([x0, x0 + d * math.cos(bearing)], np.float32)
    y = np.array([y0, y0 + d * math.sin(bearing)], np.float32)
    th = np.array([heading, 0.0], np.float32)
    dx, dy = float(x[1]) - float(x[0]), float(y[1]) - float(y[0])
    return x, y, th, math.hypot(dx, dy), math.atan2(dy, dx)


@pytest.mark.parametrize("radius_kind", ["vision", "collision"])
@pytest.mark.parametrize("offset,ambiguous", [(-0.5e-5, True), (0.5e-5, True),
                                              (-2e-5, False), (2e-5, False)])
def test_band_width_at_radius(oracle_mod, radius_kind, offset, ambiguous):
    R = 8.0 if radius_kind == "vision" else 0.5
    x, y, th, d, _ = _pair_at(R + offset, 0.3)
    assert abs((d - R) - offset) < 2e-6          # the FP32 placement kept the offset
    r = oracle_mod.oracle_sense(x, y, th, 64.0, sectors=16, agents=[0], eps_d=EPS, eps_phi=EPS)
    lo, hi = (r.nb_lo[0], r.nb_hi[0]) if R == 8.0 else (r.col_lo[0], r.col_hi[0])
    inside = d < R
    if ambiguous:
        assert (lo, hi) == (0, 1)
    else:
        assert lo == hi == int(inside)
    # the plain count follows the strict comparison whatever the band
    plain = r.n_nb[0] if R == 8.0 else r.n_col[0]
    assert plain == int(inside)


@pytest.mark.parametrize("fov_deg,v,edge_k", [(360.0, 16, 3), (360.0, 16, 0), (250.0, 16, 5),
                                              (250.0, 128, 77)])
@pytest.mark.parametrize("offset,ambiguous", [(0.5e-5, True), (-0.5e-5, True), (0.85e-5, True),
                                              (-0.85e-5, True), (2e-5, False), (-2e-5, False)])
def test_band_width_at_sector_edge(oracle_mod, fov_deg, v, edge_k, offset, ambiguous):
    """Sector edge k of a full view lies at k 2pi/v from the heading; of a
    limited view at -fov/2 + k fov/v (bearings relative to the heading)."""
    heading = 0.9
    fov = math.radians(fov_deg)
    rel_edge = edge_k * 2 * math.pi / v if fov_deg == 360.0 else -fov / 2 + edge_k * fov / v
    x, y, th, d, bearing = _pair_at(7.5, heading + rel_edge + offset, heading=heading)
    rel = math.remainder(bearing - float(np.float32(heading)), 2 * math.pi)
    measured = math.remainder(rel - rel_edge, 2 * math.pi)
    assert abs(measured - offset) < 5e-7
    kw = {} if fov_deg == 360.0 else {"fov": fov}
    r = oracle_mod.oracle_sense(x, y, th, 64.0, sectors=v, agents=[0], eps_d=EPS, eps_phi=EPS, **kw)
    strict, loose = r.dmin_strict[0], r.dmin_loose[0]
    below, above = (edge_k - 1) % v, edge_k % v
    assert r.n_nb[0] == 1
    if ambiguous:
        assert np.isinf(strict).all()
        assert np.isfinite(loose[below]) and np.isfinite(loose[above])
        assert np.count_nonzero(np.isfinite(loose)) == 2
    else:
        want = above if measured > 0 else below
        assert np.count_nonzero(np.isfinite(strict)) == 1 and np.isfinite(strict[want])
        assert np.array_equal(strict, loose)


@pytest.mark.parametrize("offset,ambiguous", [(0.5e-5, True), (-0.5e-5, True), (0.85e-5, True),
                                              (-0.85e-5, True), (2e-5, False), (-2e-5, False)])
@pytest.mark.parametrize("side", [-1, 1])
def test_band_width_at_arc_edge(oracle_mod, offset, ambiguous, side):
    """A limited view's arc ends at +-fov/2: a pair within the band of an end
    may be seen in the end sector or not seen at all."""
    heading, v = 2.2, 16
    fov = math.radians(250.0)
    rel_edge = side * fov / 2
    x, y, th, d, bearing = _pair_at(7.5, heading + rel_edge + offset, heading=heading)
    rel = math.remainder(bearing - float(np.float32(heading)), 2 * math.pi)
    measured = rel - rel_edge
    assert abs(measured - offset) < 5e-7
    r = oracle_mod.oracle_sense(x, y, th, 64.0, sectors=v, agents=[0], eps_d=EPS, eps_phi=EPS,
                                fov=fov)
    end = v - 1 if side > 0 else 0
    inside = (measured < 0) if side > 0 else (measured >= 0)
    strict, loose = r.dmin_strict[0], r.dmin_loose[0]
    assert r.n_nb[0] == 1 and np.count_nonzero(np.isfinite(loose)) == (1 if (ambiguous or inside) else 0)
    if ambiguous:
        assert np.isinf(strict).all() and np.isfinite(loose[end])
    elif inside:
        assert np.isfinite(strict[end]) and np.array_equal(strict, loose)
    else:
        assert np.isinf(strict).all() and np.isinf(loose).all()


@pytest.mark.parametrize("offset,ambiguous", [(0.85e-5, True), (-0.85e-5, True), (2e-5, False)])
def test_band_width_tag(oracle_mod, offset, ambiguous):
    """The tag oracle's bands have the flock's widths: a runner pair (channel
    0) at a 250-degree sector edge and a runner-chaser pair at the touch distance."""
    heading, v, fov = 0.4, 64, math.radians(250.0)
    rel_edge = -fov / 2 + 20 * fov / v
    x, y, th, _, bearing = _pair_at(7.5, heading + rel_edge + offset, heading=heading)
    measured = math.remainder(bearing - float(np.float32(heading)) - rel_edge, 2 * math.pi)
    assert abs(measured - offset) < 5e-7
    r = oracle_mod.oracle_sense_tag(x, y, th, 64.0, 0, radius=10.0, touch=1.0, sectors=v,
                                    agents=[0], eps_d=EPS, eps_phi=EPS, fov=fov)
    assert np.count_nonzero(np.isfinite(r.dmin_loose[0])) == (2 if ambiguous else 1)
    assert np.count_nonzero(np.isfinite(r.dmin_strict[0])) == (0 if ambiguous else 1)
    x, y, th, d, _ = _pair_at(1.0 + offset, 1.1)
    assert abs((d - 1.0) - offset) < 2e-6
    r = oracle_mod.oracle_sense_tag(x, y, th, 64.0, 1, radius=10.0, touch=1.0, sectors=v,
                                    agents=[0, 1], eps_d=EPS, eps_phi=EPS, fov=fov)
    touch = int(d < 1.0)
    for k in range(2):
        assert (r.col_lo[k], r.col_hi[k]) == ((0, 1) if ambiguous else (touch, touch))
