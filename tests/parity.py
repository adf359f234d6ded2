"""Comparison of GPU step outputs with the CPU oracle (used by the GPU tests).

Tolerances (stated once, applied everywhere):
  * EPS_D = 1e-5: a pair whose exact distance lies within 1e-5 of the vision
    range or of the collision distance may be counted either way.
  * EPS_PHI = 1e-5 rad: a pair whose exact bearing lies within 1e-5 rad of a
    sector edge may be placed in either sector.  The GPU bearing error is
    about 2e-6 rad (FP32 rotation and atan2), well inside this band.
  * Counts must lie in the oracle's [lo, hi] band (exact when no pair is
    ambiguous, which is almost always the case).
  * obs: the GPU value must lie within OBS_TOL = 1e-5 (relative to the obs
    scale of 1) of the interval spanned by the strict and loose nearest
    distances.  The GPU obs error from FP32 d^2 and sqrt is about 1e-7.
  * reward: |r_gpu - r| <= 1e-5 * max(1, |r|), r computed in FP64 from the
    counts.
  * state after the move, teacher-forced (the oracle moves the GPU's own
    pre-step state with the same actions): heading and speed bitwise equal
    (the same FP32 operations on both sides); each coordinate within
    MOVE_POS_TOL = 2^-21 plus one ulp of the oracle's value, periodically.
    The GPU's FP32 cos/sin are within 1 ulp of the correctly rounded values
    the oracle uses; scaled by a speed of at most 2 that moves the step
    s cos(theta) by at most 2^-22 before its rounding, and the sum x + step
    by at most one rounding more.  That rounding happens before the periodic
    wrap, at the magnitude of the unwrapped sum: a coordinate that wrapped
    from just above L to just above 0 carries an ulp of L, so within
    WRAP_REACH of 0 the ulp of L + WRAP_REACH is allowed.
"""
from __future__ import annotations

import numpy as np

EPS_D = 1e-5
EPS_PHI = 1e-5
OBS_TOL = 1e-5
REW_TOL = 1e-5
MOVE_POS_TOL = 2.0 ** -21
WRAP_REACH = 4.0      # above the largest step (speed at most 2, dt = 1)


def check_sense(oracle_res, obs, reward, nb, col, radius=8.0, r_nb=0.1, r_col=-1.0, label=""):
    """Assert GPU obs/reward/counts (rows = oracle_res.agents or all) are within the bands."""
    obs = np.asarray(obs, np.float64)
    reward = np.asarray(reward, np.float64)
    o = oracle_res
    stats = {}
    if nb is not None:
        nb = np.asarray(nb)
        col = np.asarray(col)
        bad = (nb < o.nb_lo) | (nb > o.nb_hi) | (col < o.col_lo) | (col > o.col_hi)
        assert not bad.any(), (f"{label}: counts outside band at rows {np.nonzero(bad)[0][:10]}: "
                               f"gpu nb {nb[bad][:5]} band [{o.nb_lo[bad][:5]}, {o.nb_hi[bad][:5]}]")
        clean = (o.nb_lo == o.nb_hi) & (o.col_lo == o.col_hi)
        assert np.array_equal(nb[clean], o.n_nb[clean]) and np.array_equal(col[clean], o.n_col[clean])
        stats["ambiguous_count_rows"] = int((~clean).sum())
        r_expect = r_nb * nb.astype(np.float64) + r_col * col.astype(np.float64)
        rerr = np.abs(reward - r_expect) / np.maximum(1.0, np.abs(r_expect))
        assert rerr.max(initial=0) <= REW_TOL, f"{label}: reward error {rerr.max()}"
        rclean = np.abs(reward[clean] - o.reward[clean]) / np.maximum(1.0, np.abs(o.reward[clean]))
        assert rclean.max(initial=0) <= REW_TOL
    else:
        rerr = np.abs(reward - o.reward) / np.maximum(1.0, np.abs(o.reward))
        amb = o.nb_lo != o.nb_hi
        amb |= o.col_lo != o.col_hi
        assert rerr[~amb].max(initial=0) <= REW_TOL, f"{label}: reward error {rerr[~amb].max()}"
    strict, loose = o.dmin_strict, o.dmin_loose
    lower = np.where(np.isfinite(strict), 1.0 - strict / radius, -OBS_TOL)
    upper = np.where(np.isfinite(loose), 1.0 - loose / radius, 0.0)
    bad = (obs < lower - OBS_TOL) | (obs > upper + OBS_TOL)
    if bad.any():
        r, k = np.nonzero(bad)
        raise AssertionError(f"{label}: obs outside band at {list(zip(r[:5], k[:5]))}: gpu "
                             f"{obs[bad][:5]} band [{lower[bad][:5]}, {upper[bad][:5]}]")
    exact = np.isfinite(strict) & (strict == loose)
    err = np.abs(obs - np.where(np.isfinite(strict), 1.0 - strict / radius, 0.0))
    stats["obs_max_err_clean"] = float(err[exact | ~np.isfinite(loose)].max(initial=0.0))
    stats["ambiguous_sector_cells"] = int((~(exact | ~np.isfinite(loose))).sum())
    return stats


def state_mismatch(a, b):
    """Indices where two FP32 state tuples differ bitwise; max ulp distance."""
    idx = np.zeros(a[0].shape[0], bool)
    ulp = 0
    for u, w in zip(a, b):
        u = np.asarray(u, np.float32)
        w = np.asarray(w, np.float32)
        d = u.view(np.int32).astype(np.int64) - w.view(np.int32).astype(np.int64)
        idx |= d != 0
        ulp = max(ulp, int(np.abs(d).max(initial=0)))
    return np.nonzero(idx)[0], ulp


def check_move(got, want, box, label=""):
    """GPU post-move state ``got`` against the oracle's move ``want`` of the same
    pre-move state (tuples x, y, heading, speed); returns the largest position
    error in units of the tolerance."""
    gx, gy, gth, gs = (np.asarray(a, np.float32) for a in got)
    wx, wy, wth, ws = (np.asarray(a, np.float32) for a in want)
    bad = np.nonzero((gth.view(np.int32) != wth.view(np.int32)) |
                     (gs.view(np.int32) != ws.view(np.int32)))[0]
    assert bad.size == 0, f"{label}: heading/speed differ at {bad[:10]}"
    worst = 0.0
    for g, w, name in ((gx, wx, "x"), (gy, wy, "y")):
        d = g.astype(np.float64) - w.astype(np.float64)
        d -= box * np.round(d / box)          # a wrap decided on either side of 0 or L
        mag = np.where(w < WRAP_REACH, np.float32(box + WRAP_REACH), np.abs(w))
        tol = MOVE_POS_TOL + np.spacing(mag.astype(np.float32)).astype(np.float64)
        r = np.abs(d) / tol
        if r.size:
            worst = max(worst, float(r.max()))
        assert (r <= 1.0).all(), (f"{label}: {name} off by {d[r > 1][:5]} at "
                                  f"{np.nonzero(r > 1)[0][:5]} (tolerance {tol[r > 1][:5]})")
        assert ((g >= 0) & (g < box)).all(), f"{label}: {name} outside [0, L)"
    return worst
