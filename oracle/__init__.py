"""CPU oracle for the flock environment step (arXiv:2207.03945, Sec. 4 and 4.1).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2207_03945_amd``) never imports it, and the two share no code.

``oracle_move`` / ``oracle_sense`` are thin ctypes wrappers round the plain C
in ``flock_oracle.c`` (all-pairs, double-precision sensing).  ``policy_forward``
is the double-precision policy network in ``policy.py``; ``rl.py`` holds the
experience-collection pieces (Gaussian action sampling, the critic, the
truncated advantage estimator); ``graph.py`` the opinion-dynamics graph
interaction.  ``oracle_move_tag`` / ``oracle_sense_tag`` are the tag
environment (runners and chasers) of Sec. 4.2.

Parity pins: every function here is pinned by ``tests/test_oracle_pins.py``,
``tests/test_oracle_rl_pins.py``, ``tests/test_oracle_tag_pins.py`` and ``tests/test_oracle_graph_pins.py``
against closed forms, brute-force lattice
counts, invariants, statistics and library densities.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from . import graph, rl  # noqa: F401
from .policy import policy_forward, xavier_limits  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flock_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fused multiply-add, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_move.argtypes = [ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float,
                                    _f32p, _f32p, _f32p, _f32p, _f32p]
        lib.oracle_move.restype = None
        opt_i32 = ctypes.c_void_p
        lib.oracle_sense.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, _f32p, _f32p, _f32p,
                                     ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_double, ctypes.c_double,
                                     _f64p, _i32p, _i32p, _f64p,
                                     opt_i32, opt_i32, opt_i32, opt_i32,
                                     ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_sense.restype = None
        lib.oracle_move_tag.argtypes = [ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, _f32p, _f32p, _f32p, _f32p, _f32p]
        lib.oracle_move_tag.restype = None
        lib.oracle_sense_tag.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, _f32p, _f32p, _f32p,
                                         ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_double, ctypes.c_double,
                                         _f64p, _i32p, _i32p, _f64p,
                                         opt_i32, opt_i32, opt_i32, opt_i32,
                                         ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_sense_tag.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def oracle_move(state, act, box, max_turn=0.2, max_dspeed=0.1, s_min=0.0, s_max=2.0):
    """Rotate / accelerate / move / wrap (Sec. 4.1).  Returns a new state tuple.

    ``state`` = (x, y, th, s) FP32 arrays; ``act`` = [n, 2] FP32 (turn, dspeed).
    """
    x, y, th, s = (np.array(a, dtype=np.float32, copy=True) for a in state)
    a = np.ascontiguousarray(act, dtype=np.float32).reshape(-1)
    n = x.shape[0]
    assert a.shape[0] == 2 * n
    _load().oracle_move(n, float(box), float(max_turn), float(max_dspeed), float(s_min),
                        float(s_max), x, y, th, s, a)
    return x, y, th, s


class SenseResult:
    """Per-agent view, counts and reward from :func:`oracle_sense`."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


TWO_PI = 2.0 * math.pi


def oracle_sense(x, y, th, box, radius=8.0, collide=0.5, sectors=16, r_nb=0.1, r_col=-1.0,
                 agents=None, eps_d=0.0, eps_phi=0.0, fov=TWO_PI) -> SenseResult:
    """View + reward for the agents in ``agents`` (all if None), all-pairs, FP64.

    Follows Sec. 4 (v sectors, nearest distance per sector), Sec. 4.1 Eq. (1)
    (sum over d_ij < d_v) and Fig. 4's collision penalty.  ``eps_d``/``eps_phi``
    request the ambiguity bands described in ``flock_oracle.c``; ``fov`` < 2 pi
    restricts the view to that arc round the heading (Sec. 5).
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    th = np.ascontiguousarray(th, dtype=np.float32)
    n = x.shape[0]
    if not 1 <= sectors <= 256:
        raise ValueError("sectors must be in [1, 256]")
    if agents is None:
        n_list, lst, lst_ptr = n, None, None
    else:
        lst = np.ascontiguousarray(agents, dtype=np.int32)
        n_list, lst_ptr = lst.shape[0], lst.ctypes.data
    obs = np.zeros((n_list, sectors), np.float64)
    n_nb = np.zeros(n_list, np.int32)
    n_col = np.zeros(n_list, np.int32)
    reward = np.zeros(n_list, np.float64)
    nb_lo = np.zeros(n_list, np.int32)
    nb_hi = np.zeros(n_list, np.int32)
    col_lo = np.zeros(n_list, np.int32)
    col_hi = np.zeros(n_list, np.int32)
    dstrict = np.zeros((n_list, sectors), np.float64)
    dloose = np.zeros((n_list, sectors), np.float64)
    if n_list > 0:
        _load().oracle_sense(n, float(box), float(radius), float(collide), int(sectors),
                             float(fov), float(r_nb), float(r_col), x, y, th, n_list, lst_ptr,
                             float(eps_d), float(eps_phi), obs, n_nb, n_col, reward,
                             nb_lo.ctypes.data, nb_hi.ctypes.data, col_lo.ctypes.data,
                             col_hi.ctypes.data, dstrict.ctypes.data, dloose.ctypes.data)
    return SenseResult(obs=obs, n_nb=n_nb, n_col=n_col, reward=reward, nb_lo=nb_lo,
                       nb_hi=nb_hi, col_lo=col_lo, col_hi=col_hi, dmin_strict=dstrict,
                       dmin_loose=dloose, agents=lst)


def oracle_move_tag(state, act, box, max_turn=0.2, s_max=2.0):
    """Tag move (Sec. 4.2): turn by the clamped first action, move at speed clamp(a1, 0, s_max)."""
    x, y, th, s = (np.array(a, dtype=np.float32, copy=True) for a in state)
    a = np.ascontiguousarray(act, dtype=np.float32).reshape(-1)
    n = x.shape[0]
    assert a.shape[0] == 2 * n
    _load().oracle_move_tag(n, float(box), float(max_turn), float(s_max), x, y, th, s, a)
    return x, y, th, s


def oracle_sense_tag(x, y, th, box, n_chasers, radius=8.0, touch=0.5, sectors=64, r_near=0.1,
                     r_caught=-1.0, r_catch=1.0, agents=None, eps_d=0.0, eps_phi=0.0,
                     fov=TWO_PI) -> SenseResult:
    """Tag view (runner channel, then chaser channel), counts and reward, all pairs, FP64.

    ``n_nb`` holds the runners within the vision range and ``n_col`` the
    touches with agents of the other type (fields named as for the flock).
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    th = np.ascontiguousarray(th, dtype=np.float32)
    n = x.shape[0]
    if not 1 <= sectors <= 256:
        raise ValueError("sectors must be in [1, 256]")
    if agents is None:
        n_list, lst, lst_ptr = n, None, None
    else:
        lst = np.ascontiguousarray(agents, dtype=np.int32)
        n_list, lst_ptr = lst.shape[0], lst.ctypes.data
    w = 2 * sectors
    obs = np.zeros((n_list, w), np.float64)
    n_nb = np.zeros(n_list, np.int32)
    n_col = np.zeros(n_list, np.int32)
    reward = np.zeros(n_list, np.float64)
    nb_lo, nb_hi, col_lo, col_hi = (np.zeros(n_list, np.int32) for _ in range(4))
    dstrict = np.zeros((n_list, w), np.float64)
    dloose = np.zeros((n_list, w), np.float64)
    if n_list > 0:
        _load().oracle_sense_tag(n, int(n_chasers), float(box), float(radius), float(touch),
                                 int(sectors), float(fov), float(r_near), float(r_caught),
                                 float(r_catch), x, y, th, n_list, lst_ptr, float(eps_d),
                                 float(eps_phi), obs, n_nb, n_col, reward, nb_lo.ctypes.data,
                                 nb_hi.ctypes.data, col_lo.ctypes.data, col_hi.ctypes.data,
                                 dstrict.ctypes.data, dloose.ctypes.data)
    return SenseResult(obs=obs, n_nb=n_nb, n_col=n_col, reward=reward, nb_lo=nb_lo,
                       nb_hi=nb_hi, col_lo=col_lo, col_hi=col_hi, dmin_strict=dstrict,
                       dmin_loose=dloose, agents=lst)


def observation(sense, speed=None):
    """The agent's observation: its v-sector view, then its speed when given.

    Sec. 4.1 describes the flock observation as the view followed by the
    agent's current speed (129 = 128 sectors + speed).
    """
    if speed is None:
        return sense.obs
    rows = slice(None) if sense.agents is None else sense.agents
    return np.concatenate([sense.obs, np.asarray(speed, np.float64)[rows, None]], axis=1)


def oracle_step(state, act, box, radius=8.0, collide=0.5, sectors=16, r_nb=0.1, r_col=-1.0,
                max_turn=0.2, max_dspeed=0.1, s_min=0.0, s_max=2.0, eps_d=0.0, eps_phi=0.0,
                agents=None, fov=TWO_PI):
    """One full step (Sec. 4.1 order): move every agent, then sense."""
    new_state = oracle_move(state, act, box, max_turn, max_dspeed, s_min, s_max)
    sense = oracle_sense(new_state[0], new_state[1], new_state[2], box, radius, collide,
                         sectors, r_nb, r_col, agents=agents, eps_d=eps_d, eps_phi=eps_phi,
                         fov=fov)
    return new_state, sense
