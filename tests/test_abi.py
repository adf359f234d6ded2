"""C-ABI checks that need no GPU: the library loads, exports every function
include/flockenv.h declares, and its validation layer rejects bad arguments
before any HIP call."""
from __future__ import annotations

import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flockenv.h")

flock = pytest.importorskip("paper_2207_03945_amd")
from paper_2207_03945_amd import flockenv as fe  # noqa: E402


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][A-Za-z0-9_ \*]*?\b([a-z_]+[a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted({n for n in names if n not in ("defined",)})


def test_exports_every_declared_symbol():
    lib = fe.lib()
    names = declared_functions()
    assert len(names) >= 30, names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def _bytes(**kw):
    base = dict(n_agents=256, box=64.0)
    base.update(kw)
    return fe.lib().env_workspace_bytes(ctypes.byref(fe.Params(**base).c()))


@pytest.mark.parametrize("kw", [
    dict(n_agents=-1), dict(n_agents=(1 << 26) + 1), dict(box=0.0), dict(box=math.inf),
    dict(box=math.nan), dict(radius=0.0), dict(radius=32.0), dict(radius=40.0),
    dict(collide=-0.1), dict(collide=9.0), dict(sectors=0), dict(sectors=257),
    dict(r_nb=math.nan), dict(max_turn=-0.1), dict(max_dspeed=math.inf), dict(s_min=-1.0),
    dict(s_min=3.0, s_max=2.0), dict(cell_reach=3), dict(cell_reach=-1), dict(flags=8),
    dict(flags=16), dict(flags=4, n_chasers=-1), dict(flags=4, n_chasers=300),
    dict(flags=4, r_catch=math.nan), dict(flags=4, sectors=129), dict(fov=-0.1), dict(fov=6.3), dict(fov=math.nan), dict(fov=math.inf),
])
def test_invalid_params_rejected(kw):
    assert _bytes(**kw) == 0
    assert fe.last_error() != ""


@pytest.mark.parametrize("kw", [dict(), dict(n_agents=0), dict(sectors=1), dict(sectors=256),
                                dict(radius=31.99), dict(collide=0.0), dict(cell_reach=2),
                                dict(flags=1), dict(flags=2), dict(flags=3),
                                dict(fov=math.radians(250.0)), dict(fov=1e-3),
                                dict(fov=float(np.float32(2 * math.pi))),
                                dict(flags=4, n_chasers=23, sectors=64),
                                dict(flags=6, n_chasers=0, sectors=128)])
def test_valid_params_accepted(kw):
    assert _bytes(**kw) > 0


def _create(nbytes=None, ws=1 << 20, **kw):
    p = fe.Params(**{**dict(n_agents=256, box=64.0), **kw}).c()
    need = fe.lib().env_workspace_bytes(ctypes.byref(p))
    h = ctypes.c_void_p()
    rc = fe.lib().env_create(ctypes.byref(p), ws, need if nbytes is None else nbytes, ctypes.byref(h))
    return rc, h, need


def test_create_errors_without_gpu():
    lib = fe.lib()
    rc, _, _ = _create(ws=None)
    assert rc == fe.ENV_EINVAL
    rc, _, _ = _create(ws=(1 << 20) + 8)
    assert rc == fe.ENV_EINVAL and "aligned" in fe.last_error()
    rc, _, need = _create(nbytes=100)
    assert rc == fe.ENV_ENOMEM
    # a valid bind makes no HIP call, so it succeeds on a host address
    rc, h, _ = _create()
    assert rc == fe.ENV_OK
    nx, ny, reach = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    cw, ch = ctypes.c_float(), ctypes.c_float()
    assert lib.env_geometry(h, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(reach),
                            ctypes.byref(cw), ctypes.byref(ch)) == 0
    assert (nx.value, ny.value, reach.value) == (7, 28, 1) and cw.value > 8.0
    assert lib.env_geometry(h, None, None, None, None, None) == 0
    assert lib.env_geometry(None, None, None, None, None, None) == fe.ENV_EINVAL
    # call order: step / reset / counts before their preconditions
    assert lib.env_step(h, 1 << 20, 1 << 20, 1 << 20, None) == fe.ENV_ESTATE
    assert lib.env_reset(h, 1 << 20, None) == fe.ENV_ESTATE
    assert lib.env_get_counts(h, 1 << 20, 1 << 20, None) == fe.ENV_ESTATE
    assert lib.env_get_returns(h, 1 << 20, None) == fe.ENV_ESTATE
    assert lib.env_get_state(h, 1 << 20, 1 << 20, 1 << 20, 1 << 20, None) == fe.ENV_ESTATE
    assert lib.env_set_state(h, None, None, None, None, None) == fe.ENV_EINVAL
    lib.env_destroy(h)
    assert lib.env_step(None, None, None, None, None) == fe.ENV_EINVAL


def _geometry(h):
    nx, ny, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    cw, ch = ctypes.c_float(), ctypes.c_float()
    assert fe.lib().env_geometry(h, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(r),
                                 ctypes.byref(cw), ctypes.byref(ch)) == 0
    return nx.value, ny.value, r.value, cw.value, ch.value


@pytest.mark.parametrize("box,ncell,reach", [(64.0, 7, 1), (316.0, 39, 1), (1000.0, 124, 1),
                                             (20.0, 1, 0), (24.0, 1, 0), (24.5, 3, 1)])
def test_geometry(box, ncell, reach):
    rc, h, _ = _create(n_agents=50000, box=box)
    assert rc == 0
    nx, ny, r, cw, ch = _geometry(h)
    assert (nx, r) == (ncell, reach)
    if ncell > 1:
        # every column is wider than the vision range plus the rounding margin
        assert box / ncell >= 8.0 + 4 * box * 2.0 ** -23
        assert ny == 4 * nx and cw == np.float32(box / nx) and ch == np.float32(box / ny)
    else:
        assert ny == 1
    fe.lib().env_destroy(h)


def test_reach_two_geometry():
    rc, h, _ = _create(n_agents=50000, box=160.0, cell_reach=2)
    nx, ny, r, cw, ch = _geometry(h)
    assert r == 2 and 160.0 / nx >= 4.0 and ny == 4 * nx
    fe.lib().env_destroy(h)


def test_batch_validation_without_gpu():
    lib = fe.lib()
    arr = (ctypes.c_void_p * 2)()
    pp = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    assert lib.env_batch_workspace_bytes(pp, 0) == 0
    assert lib.env_batch_workspace_bytes(pp, 2) == 0          # NULL envs
    rc1, h1, _ = _create(sectors=16)
    rc2, h2, _ = _create(sectors=8)
    arr[0], arr[1] = h1.value, h2.value
    assert lib.env_batch_workspace_bytes(pp, 2) == 0 and "sectors" in fe.last_error()
    b = ctypes.c_void_p()
    assert lib.env_batch_create(pp, 2, 1 << 20, 1 << 30, ctypes.byref(b)) == fe.ENV_EINVAL
    rc3, h3, _ = _create(sectors=16, flags=fe.ENV_FLAG_SPEED_OBS)
    arr[1] = h3.value
    assert lib.env_batch_workspace_bytes(pp, 2) == 0 and "SPEED_OBS" in fe.last_error()
    rc5, h5, _ = _create(sectors=16, flags=fe.ENV_FLAG_TAG, n_chasers=10)
    arr[1] = h5.value   # tag and flock envs do not mix
    assert lib.env_batch_workspace_bytes(pp, 2) == 0 and "TAG" in fe.last_error()
    lib.env_destroy(h5)
    rc4, h4, _ = _create(sectors=16, fov=math.radians(250.0))
    arr[1] = h4.value   # fields of view may differ within a batch
    assert lib.env_batch_workspace_bytes(pp, 2) > 0
    arr[1] = h1.value
    assert lib.env_batch_workspace_bytes(pp, 2) > 0
    # envs not reset yet
    assert lib.env_batch_create(pp, 2, 1 << 20, 1 << 30, ctypes.byref(b)) == fe.ENV_ESTATE
    for h in (h1, h2, h3, h4):
        lib.env_destroy(h)


def test_policy_and_server_validation_without_gpu():
    lib = fe.lib()
    assert lib.pol_workspace_bytes(16, 64) > 0
    assert lib.pol_workspace_bytes(33, 64) > lib.pol_workspace_bytes(32, 64) == lib.pol_workspace_bytes(16, 64)
    assert lib.pol_workspace_bytes(257, 64) > lib.pol_workspace_bytes(129, 64) > 0
    for bad in ((0, 64), (258, 64), (16, 32)):
        assert lib.pol_workspace_bytes(*bad) == 0
    h = ctypes.c_void_p()
    assert lib.pol_create(None, 16, 64, 0.2, 0.1, 1 << 20, 1 << 20, None, ctypes.byref(h)) == fe.ENV_EINVAL
    w = (ctypes.c_float * 10000)()
    assert lib.pol_create(w, 16, 64, -0.2, 0.1, 1 << 20, 1 << 20, None, ctypes.byref(h)) == fe.ENV_EINVAL
    assert lib.pol_create(w, 16, 64, 0.2, 0.1, 1 << 20, 10, None, ctypes.byref(h)) == fe.ENV_ENOMEM
    assert lib.pol_forward(None, None, 0, None, None) == fe.ENV_EINVAL
    s = ctypes.c_void_p()
    assert lib.srv_create(None, 1 << 20, 4, None, None, ctypes.byref(s)) == fe.ENV_EINVAL
    assert lib.srv_tick(None, None, None) == fe.ENV_EINVAL
    p = fe.Params(n_agents=5000, box=316.0)
    small = fe.Params(n_agents=500, box=90.0)
    assert fe.request_bytes(p) > fe.request_bytes(small) > 0
    assert fe.request_bytes(fe.Params(n_agents=10, box=10.0)) == 0


def test_sweep_lanes_validation_without_gpu():
    lib = fe.lib()
    rc, h, _ = _create()
    assert rc == fe.ENV_OK
    for bad in (2, 3, 8, 128, -1):
        assert lib.env_set_sweep_lanes(h, bad) == fe.ENV_EINVAL
    for ok in (0, 1, 4, 16, 64):
        assert lib.env_set_sweep_lanes(h, ok) == fe.ENV_OK
    assert lib.env_set_sweep_lanes(None, 1) == fe.ENV_EINVAL
    assert lib.env_batch_set_sweep_lanes(None, 1) == fe.ENV_EINVAL
    lib.env_destroy(h)


def test_rl_validation_without_gpu():
    lib = fe.lib()
    buf = 1 << 20
    assert lib.rl_gae(0, 10, 0.99, 0.95, buf, buf, buf, buf, None) == fe.ENV_EINVAL
    assert lib.rl_gae(4, -1, 0.99, 0.95, buf, buf, buf, buf, None) == fe.ENV_EINVAL
    assert lib.rl_gae(4, 10, 1.5, 0.95, buf, buf, buf, buf, None) == fe.ENV_EINVAL
    assert lib.rl_gae(4, 10, 0.99, -0.1, buf, buf, buf, buf, None) == fe.ENV_EINVAL
    assert lib.rl_gae(4, 10, math.nan, 0.9, buf, buf, buf, buf, None) == fe.ENV_EINVAL
    assert lib.rl_gae(4, 10, 0.99, 0.95, None, buf, buf, buf, None) == fe.ENV_EINVAL
    assert lib.rl_gae(4, 0, 0.99, 0.95, None, None, None, None, None) == fe.ENV_OK
    h = ctypes.c_void_p()
    w = (ctypes.c_float * 20000)()
    assert lib.pol_create_value(None, 16, 64, 1 << 20, 1 << 20, None, ctypes.byref(h)) == fe.ENV_EINVAL
    assert lib.pol_create_value(w, 300, 64, 1 << 20, 1 << 20, None, ctypes.byref(h)) == fe.ENV_EINVAL
    assert lib.pol_create_value(w, 16, 64, 1 << 20, 10, None, ctypes.byref(h)) == fe.ENV_ENOMEM
    assert lib.pol_value(None, None, 0, None, None) == fe.ENV_EINVAL
    assert lib.pol_sample(None, None, 0, None, None, None, None, None) == fe.ENV_EINVAL
    assert lib.env_rollout(None, None, 4, None, None, None, None, None, None, None) == fe.ENV_EINVAL


def test_graph_validation_without_gpu():
    lib = fe.lib()
    b = 1 << 20
    assert lib.gr_opinion_step(-1, 0, b, b, b, 0.3, 0.5, b, b + 64, 0, None) == fe.ENV_EINVAL
    assert lib.gr_opinion_step(1 << 31, 0, b, b, b, 0.3, 0.5, b, b + 64, 0, None) == fe.ENV_EINVAL
    assert lib.gr_opinion_step(10, -1, b, b, b, 0.3, 0.5, b, b + 64, 0, None) == fe.ENV_EINVAL
    assert lib.gr_opinion_step(10, 5, b, b, b, math.nan, 0.5, b, b + 64, 0, None) == fe.ENV_EINVAL
    assert lib.gr_opinion_step(10, 5, b, b, b, 0.3, 0.5, b, b + 64, 2, None) == fe.ENV_EINVAL
    assert lib.gr_opinion_step(10, 5, None, b, b, 0.3, 0.5, b, b + 64, 0, None) == fe.ENV_EINVAL
    assert lib.gr_opinion_step(10, 5, b, None, b, 0.3, 0.5, b, b + 64, 0, None) == fe.ENV_EINVAL
    assert lib.gr_opinion_step(10, 5, b, b, b, 0.3, 0.5, b, b, 0, None) == fe.ENV_EINVAL
    assert lib.gr_opinion_step(0, 0, None, None, None, 0.3, 0.5, None, None, 0, None) == fe.ENV_OK


def test_obs_dim():
    assert fe.Params(n_agents=4, box=64.0, sectors=128).obs_dim == 128
    assert fe.Params(n_agents=4, box=64.0, sectors=128, flags=fe.ENV_FLAG_SPEED_OBS).obs_dim == 129
    assert fe.Params(n_agents=4, box=64.0, flags=3).obs_dim == 17
    assert fe.Params(n_agents=4, box=64.0, sectors=64, flags=fe.ENV_FLAG_TAG).obs_dim == 128
    assert fe.Params(n_agents=4, box=64.0, sectors=64, flags=6).obs_dim == 129


def test_missing_library_raises(tmp_path, monkeypatch):
    monkeypatch.setattr(fe, "_lib", None)
    monkeypatch.setattr(fe, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        fe.lib()
