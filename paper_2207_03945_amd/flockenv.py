"""ctypes binding of ``libflockenv.so`` (declared in include/flockenv.h).

Argument marshalling only: every step of the environment runs in the HIP
kernels behind the C ABI.  PyTorch provides device memory (workspaces and the
act/obs/reward tensors) and streams.  There is no CPU fallback: if the built
library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflockenv.so")

ENV_OK, ENV_EINVAL, ENV_ENOMEM, ENV_ESTATE, ENV_EHIP, ENV_EAGAIN, ENV_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
ENV_FLAG_COUNTS = 1
ENV_FLAG_SPEED_OBS = 2
ENV_FLAG_TAG = 4

_CODES = {ENV_EINVAL: "ENV_EINVAL", ENV_ENOMEM: "ENV_ENOMEM", ENV_ESTATE: "ENV_ESTATE",
          ENV_EHIP: "ENV_EHIP", ENV_EAGAIN: "ENV_EAGAIN", ENV_ENOTFOUND: "ENV_ENOTFOUND"}


class FlockError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class EnvParams(ctypes.Structure):
    _fields_ = [("n_agents", ctypes.c_int32), ("box", ctypes.c_float), ("radius", ctypes.c_float),
                ("collide", ctypes.c_float), ("sectors", ctypes.c_int32), ("r_nb", ctypes.c_float),
                ("r_col", ctypes.c_float), ("max_turn", ctypes.c_float),
                ("max_dspeed", ctypes.c_float), ("s_min", ctypes.c_float), ("s_max", ctypes.c_float),
                ("cell_reach", ctypes.c_int32), ("flags", ctypes.c_int32), ("fov", ctypes.c_float),
                ("n_chasers", ctypes.c_int32), ("r_catch", ctypes.c_float)]


@dataclass
class Params:
    """Flock parameters (Sec. 4.1); defaults are the paper-scale workload's constants."""
    n_agents: int
    box: float
    radius: float = 8.0
    collide: float = 0.5
    sectors: int = 16
    r_nb: float = 0.1
    r_col: float = -1.0
    max_turn: float = 0.2
    max_dspeed: float = 0.1
    s_min: float = 0.0
    s_max: float = 2.0
    cell_reach: int = 0
    flags: int = 0
    fov: float = 0.0   # view arc in radians; 0 = full circle
    n_chasers: int = 0  # tag envs (ENV_FLAG_TAG): agents 0 .. n_chasers-1 chase
    r_catch: float = 1.0  # tag: chaser reward per runner touched

    @property
    def obs_dim(self) -> int:
        """Length of a view row: the sectors (two channels for tag), then the speed."""
        channels = 2 if self.flags & ENV_FLAG_TAG else 1
        return channels * self.sectors + (1 if self.flags & ENV_FLAG_SPEED_OBS else 0)

    def c(self) -> EnvParams:
        return EnvParams(*[getattr(self, f.name) for f in fields(self)])


_lib = None
_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)


def lib():
    """Load the HIP library; raise ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2207_03945_amd/build.py "
                          "(or __graft_entry__.build()) first; there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    ep = ctypes.POINTER(EnvParams)
    sig = {
        "env_last_error": (ctypes.c_char_p, []),
        "env_workspace_bytes": (ctypes.c_size_t, [ep]),
        "env_create": (ctypes.c_int, [ep, _P, ctypes.c_size_t, _PP]),
        "env_destroy": (None, [_P]),
        "env_geometry": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_float)]),
        "env_set_state": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
        "env_get_state": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
        "env_reset": (ctypes.c_int, [_P, _P, _P]),
        "env_step": (ctypes.c_int, [_P, _P, _P, _P, _P]),
        "env_get_counts": (ctypes.c_int, [_P, _P, _P, _P]),
        "env_get_returns": (ctypes.c_int, [_P, _P, _P]),
        "env_set_returns": (ctypes.c_int, [_P, _P, _P]),
        "env_static_scratch_bytes": (ctypes.c_size_t, []),
        "env_step_static": (ctypes.c_int, [_P, _P, _P, _P, _P]),
        "env_batch_workspace_bytes": (ctypes.c_size_t, [_PP, ctypes.c_int]),
        "env_batch_create": (ctypes.c_int, [_PP, ctypes.c_int, _P, ctypes.c_size_t, _PP]),
        "env_batch_destroy": (None, [_P]),
        "env_batch_offsets": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
        "env_set_sweep_lanes": (ctypes.c_int, [_P, ctypes.c_int]),
        "env_batch_set_sweep_lanes": (ctypes.c_int, [_P, ctypes.c_int]),
        "env_batch_get_sweep_lanes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
        "env_batch_set_policy_fusion": (ctypes.c_int, [_P, ctypes.c_int]),
        "env_batch_set_strip_wait": (ctypes.c_int, [_P, ctypes.c_int]),
        "env_step_batched": (ctypes.c_int, [_P, _P, _P, _P, _P]),
        "env_batch_run": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P]),
        "env_batch_capture": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P]),
        "env_step_batched_timed": (ctypes.c_int, [_P, _P, _P, _P, _P,
                                                  ctypes.POINTER(ctypes.c_float)]),
        "pol_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
        "pol_create": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                      ctypes.c_float, _P, ctypes.c_size_t, _P, _PP]),
        "pol_destroy": (None, [_P]),
        "pol_forward": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
        "env_step_policy": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
        "pol_create_value": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_size_t,
                                            _P, _PP]),
        "pol_value": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P]),
        "pol_sample": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P, _P, _P, _P]),
        "env_rollout": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P]),
        "env_rollout_tag": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P]),
        "env_step_policy_tag": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
        "rl_gae": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                                  _P, _P, _P, _P, _P]),
        "gr_opinion_step": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, _P, _P, _P,
                                           ctypes.c_float, ctypes.c_float, _P, _P, ctypes.c_int,
                                           _P]),
        "srv_create": (ctypes.c_int, [_P, ctypes.c_size_t, ctypes.c_int, _P, _P, _PP]),
        "srv_destroy": (None, [_P]),
        "srv_submit": (ctypes.c_int, [_P, ep, _P, _P, _P, _P, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int64)]),
        "srv_tick": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int64)]),
        "srv_poll": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]),
        "srv_result": (ctypes.c_int, [_P, ctypes.c_int64, _P, ctypes.c_int64]),
        "srv_request_bytes": (ctypes.c_size_t, [ep]),
    }
    for name, (res, args) in sig.items():
        if not hasattr(L, name):
            continue
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return lib().env_last_error().decode()


def check(rc: int) -> int:
    if rc != ENV_OK:
        raise FlockError(rc, last_error())
    return rc


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream=None) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def _dev_f32(t, shape, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def workspace_bytes(params: Params) -> int:
    return int(lib().env_workspace_bytes(ctypes.byref(params.c())))


class Env:
    """One flock environment bound to a torch-allocated device workspace."""

    def __init__(self, params: Params, device="cuda"):
        self.params = params
        self.n = params.n_agents
        self.v = params.sectors
        self.d = params.obs_dim
        cp = params.c()
        nbytes = lib().env_workspace_bytes(ctypes.byref(cp))
        if nbytes == 0:
            raise FlockError(ENV_EINVAL, last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(lib().env_create(ctypes.byref(cp), self.workspace.data_ptr(), nbytes, ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.env_destroy(h)
            self.handle = None

    def geometry(self):
        """(ncx, ncy, reach, cell_w, cell_h): columns, rows per column, stencil
        half-width in columns, column width, row height."""
        nx, ny, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        cw, ch = ctypes.c_float(), ctypes.c_float()
        check(lib().env_geometry(self.handle, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(r),
                                 ctypes.byref(cw), ctypes.byref(ch)))
        return nx.value, ny.value, r.value, cw.value, ch.value

    def set_sweep_lanes(self, lanes: int):
        """Lanes per agent in the neighbour sweep (1, 4, 16, 64; 0 = automatic)."""
        check(lib().env_set_sweep_lanes(self.handle, int(lanes)))

    def set_state(self, x, y, th, s, stream=None):
        for t, nm in ((x, "x"), (y, "y"), (th, "th"), (s, "s")):
            _dev_f32(t, (self.n,), nm)
        check(lib().env_set_state(self.handle, _ptr(x), _ptr(y), _ptr(th), _ptr(s), _stream(stream)))

    def get_state(self, stream=None):
        out = [torch.empty(self.n, dtype=torch.float32, device=self.workspace.device) for _ in range(4)]
        check(lib().env_get_state(self.handle, *[_ptr(t) for t in out], _stream(stream)))
        return tuple(out)

    def reset(self, obs=None, stream=None):
        if obs is None:
            obs = torch.empty(self.n, self.d, dtype=torch.float32, device=self.workspace.device)
        _dev_f32(obs, (self.n, self.d), "obs")
        check(lib().env_reset(self.handle, _ptr(obs), _stream(stream)))
        return obs

    def step(self, act, obs=None, reward=None, stream=None):
        dev = self.workspace.device
        if obs is None:
            obs = torch.empty(self.n, self.d, dtype=torch.float32, device=dev)
        if reward is None:
            reward = torch.empty(self.n, dtype=torch.float32, device=dev)
        _dev_f32(act, (self.n, 2), "act")
        _dev_f32(obs, (self.n, self.d), "obs")
        _dev_f32(reward, (self.n,), "reward")
        check(lib().env_step(self.handle, _ptr(act), _ptr(obs), _ptr(reward), _stream(stream)))
        return obs, reward

    def step_static(self, act, obs=None, reward=None, stream=None):
        """As :meth:`step`, with the step's scratch in the library's static
        device array (env_step_static): nothing is allocated by the call."""
        dev = self.workspace.device
        if obs is None:
            obs = torch.empty(self.n, self.d, dtype=torch.float32, device=dev)
        if reward is None:
            reward = torch.empty(self.n, dtype=torch.float32, device=dev)
        _dev_f32(act, (self.n, 2), "act")
        _dev_f32(obs, (self.n, self.d), "obs")
        _dev_f32(reward, (self.n,), "reward")
        check(lib().env_step_static(self.handle, _ptr(act), _ptr(obs), _ptr(reward),
                                    _stream(stream)))
        return obs, reward

    def counts(self, stream=None):
        dev = self.workspace.device
        nb = torch.empty(self.n, dtype=torch.int32, device=dev)
        col = torch.empty(self.n, dtype=torch.int32, device=dev)
        check(lib().env_get_counts(self.handle, _ptr(nb), _ptr(col), _stream(stream)))
        return nb, col

    def returns(self, stream=None):
        ret = torch.empty(self.n, dtype=torch.float64, device=self.workspace.device)
        check(lib().env_get_returns(self.handle, _ptr(ret), _stream(stream)))
        return ret

    def set_returns(self, ret, stream=None):
        """Restore per-agent FP64 returns (after reset, when resuming an episode)."""
        if not (isinstance(ret, torch.Tensor) and ret.is_cuda and ret.dtype == torch.float64
                and ret.is_contiguous() and tuple(ret.shape) == (self.n,)):
            raise TypeError(f"ret must be a contiguous float64 CUDA tensor of shape ({self.n},)")
        check(lib().env_set_returns(self.handle, _ptr(ret), _stream(stream)))


class Batch:
    """Several envs stepped together; rows of env k are offsets[k]:offsets[k+1]."""

    def __init__(self, envs):
        self.envs = list(envs)
        arr = (ctypes.c_void_p * len(self.envs))(*[e.handle.value for e in self.envs])
        self._arr = arr
        pp = ctypes.cast(arr, _PP)
        nbytes = lib().env_batch_workspace_bytes(pp, len(self.envs))
        if nbytes == 0:
            raise FlockError(ENV_EINVAL, last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.envs[0].workspace.device)
        h = ctypes.c_void_p()
        check(lib().env_batch_create(pp, len(self.envs), self.workspace.data_ptr(), nbytes,
                                     ctypes.byref(h)))
        self.handle = h
        off = (ctypes.c_int64 * (len(self.envs) + 1))()
        check(lib().env_batch_offsets(self.handle, off))
        self.offsets = list(off)
        self.n = self.offsets[-1]
        self.v = self.envs[0].v
        self.d = self.envs[0].d

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.env_batch_destroy(h)
            self.handle = None

    def set_sweep_lanes(self, lanes: int):
        """Lanes per agent in the batched sweep (1, 4, 16, 64; 0 = automatic)."""
        check(lib().env_batch_set_sweep_lanes(self.handle, int(lanes)))

    def set_policy_fusion(self, on: bool):
        """Run the policy inside the view sweep in step_policy / rollout (off by default)."""
        check(lib().env_batch_set_policy_fusion(self.handle, 1 if on else 0))

    def set_strip_wait(self, polls: int):
        """Bound on the strip sort's look-back wait (polling rounds; 0: every
        strip counts the agents before it itself).  Results do not depend on it."""
        check(lib().env_batch_set_strip_wait(self.handle, int(polls)))

    @property
    def sweep_lanes(self) -> int:
        v = ctypes.c_int32()
        check(lib().env_batch_get_sweep_lanes(self.handle, ctypes.byref(v)))
        return v.value

    def step(self, act, obs, reward, stream=None):
        _dev_f32(act, (self.n, 2), "act")
        _dev_f32(obs, (self.n, self.d), "obs")
        _dev_f32(reward, (self.n,), "reward")
        check(lib().env_step_batched(self.handle, _ptr(act), _ptr(obs), _ptr(reward), _stream(stream)))

    def step_timed(self, act, obs, reward, stream=None):
        """One step; returns (move, scan, scatter, sweep) durations in ms (HIP events)."""
        _dev_f32(act, (self.n, 2), "act")
        _dev_f32(obs, (self.n, self.d), "obs")
        _dev_f32(reward, (self.n,), "reward")
        ms = (ctypes.c_float * 4)()
        check(lib().env_step_batched_timed(self.handle, _ptr(act), _ptr(obs), _ptr(reward),
                                           _stream(stream), ms))
        return tuple(ms)

    def capture(self, k_steps, act, obs, reward, stream):
        """Capture the k-step graph ``run`` replays, without launching it."""
        _dev_f32(act, (k_steps, self.n, 2), "act")
        _dev_f32(obs, (self.n, self.d), "obs")
        _dev_f32(reward, (k_steps, self.n), "reward")
        check(lib().env_batch_capture(self.handle, k_steps, _ptr(act), _ptr(obs), _ptr(reward),
                                      _stream(stream)))

    def run(self, k_steps, act, obs, reward, stream):
        """k_steps steps replayed from a HIP graph; ``stream`` must not be the null stream."""
        _dev_f32(act, (k_steps, self.n, 2), "act")
        _dev_f32(obs, (self.n, self.d), "obs")
        _dev_f32(reward, (k_steps, self.n), "reward")
        check(lib().env_batch_run(self.handle, k_steps, _ptr(act), _ptr(obs), _ptr(reward),
                                  _stream(stream)))

    def rollout(self, policy, steps, obs, act, reward, logp=None, eps=None, log_std=None,
                stream=None):
        """`steps` closed-loop steps into rollout buffers (env_rollout of the C ABI).

        obs [steps + 1, G, d] (block 0 = current view), act [steps, G, 2],
        reward [steps, G], logp [steps, G] or None; eps [steps, G, 2] standard
        normals and log_std (2 floats) for Gaussian sampling, or None for the
        mean action.  ``stream`` must be a non-default torch stream.
        """
        _dev_f32(obs, (steps + 1, self.n, self.d), "obs")
        _dev_f32(act, (steps, self.n, 2), "act")
        _dev_f32(reward, (steps, self.n), "reward")
        if logp is not None:
            _dev_f32(logp, (steps, self.n), "logp")
        ls = None
        if eps is not None:
            _dev_f32(eps, (steps, self.n, 2), "eps")
            ls = (ctypes.c_float * 2)(*[float(x) for x in log_std])
        check(lib().env_rollout(self.handle, policy.handle, int(steps), ls, _ptr(eps), _ptr(obs),
                                _ptr(act), _ptr(logp), _ptr(reward), _stream(stream)))

    def rollout_tag(self, runner, chaser, steps, obs, act, reward, logp=None, eps=None,
                    log_std=None, stream=None):
        """Tag rollout: as ``rollout`` with a policy per type; log_std = 4 floats
        (runner's two, then the chaser's)."""
        _dev_f32(obs, (steps + 1, self.n, self.d), "obs")
        _dev_f32(act, (steps, self.n, 2), "act")
        _dev_f32(reward, (steps, self.n), "reward")
        if logp is not None:
            _dev_f32(logp, (steps, self.n), "logp")
        ls = None
        if eps is not None:
            _dev_f32(eps, (steps, self.n, 2), "eps")
            ls = (ctypes.c_float * 4)(*[float(x) for x in log_std])
        check(lib().env_rollout_tag(self.handle, runner.handle, chaser.handle, int(steps), ls,
                                    _ptr(eps), _ptr(obs), _ptr(act), _ptr(logp), _ptr(reward),
                                    _stream(stream)))

    def step_policy_tag(self, runner, chaser, act, obs, reward, stream=None):
        _dev_f32(act, (self.n, 2), "act")
        _dev_f32(obs, (self.n, self.d), "obs")
        _dev_f32(reward, (self.n,), "reward")
        check(lib().env_step_policy_tag(self.handle, runner.handle, chaser.handle, _ptr(act),
                                        _ptr(obs), _ptr(reward), _stream(stream)))

    def step_policy(self, policy, act, obs, reward, stream=None):
        _dev_f32(act, (self.n, 2), "act")
        _dev_f32(obs, (self.n, self.d), "obs")
        _dev_f32(reward, (self.n,), "reward")
        check(lib().env_step_policy(self.handle, policy.handle, _ptr(act), _ptr(obs), _ptr(reward),
                                    _stream(stream)))


def pack_policy_weights(weights, biases):
    """Flatten W1, b1, W2, b2, W3, b3 (fan_in x fan_out, row-major) into one FP32 host array."""
    import numpy as np
    parts = []
    for w, b in zip(weights, biases):
        parts.append(np.ascontiguousarray(w, dtype=np.float32).ravel())
        parts.append(np.ascontiguousarray(b, dtype=np.float32).ravel())
    return np.ascontiguousarray(np.concatenate(parts), dtype=np.float32)


class Policy:
    """Shared policy network (in -> 64 -> 64 -> 2, tanh) in BF16 on MFMA."""

    def __init__(self, weights, biases, max_turn=0.2, max_dspeed=0.1, device="cuda", stream=None):
        in_dim, hidden = weights[0].shape
        self.in_dim, self.hidden = int(in_dim), int(hidden)
        self._host = pack_policy_weights(weights, biases)
        nbytes = lib().pol_workspace_bytes(self.in_dim, self.hidden)
        if nbytes == 0:
            raise FlockError(ENV_EINVAL, last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(lib().pol_create(self._host.ctypes.data, self.in_dim, self.hidden, max_turn,
                               max_dspeed, self.workspace.data_ptr(), nbytes, _stream(stream),
                               ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.pol_destroy(h)
            self.handle = None

    def forward(self, obs, act=None, stream=None):
        n = obs.shape[0]
        if act is None:
            act = torch.empty(n, 2, dtype=torch.float32, device=obs.device)
        _dev_f32(obs, (n, self.in_dim), "obs")
        _dev_f32(act, (n, 2), "act")
        check(lib().pol_forward(self.handle, _ptr(obs), n, _ptr(act), _stream(stream)))
        return act


    def sample(self, obs, eps, log_std, act=None, logp=None, stream=None):
        """Gaussian actions round the mean: (act [n, 2], logp [n])."""
        n = obs.shape[0]
        if act is None:
            act = torch.empty(n, 2, dtype=torch.float32, device=obs.device)
        if logp is None:
            logp = torch.empty(n, dtype=torch.float32, device=obs.device)
        _dev_f32(obs, (n, self.in_dim), "obs")
        _dev_f32(eps, (n, 2), "eps")
        _dev_f32(act, (n, 2), "act")
        _dev_f32(logp, (n,), "logp")
        ls = (ctypes.c_float * 2)(*[float(x) for x in log_std])
        check(lib().pol_sample(self.handle, _ptr(obs), n, ls, _ptr(eps), _ptr(act), _ptr(logp),
                               _stream(stream)))
        return act, logp


class Critic:
    """Value network (in -> 64 -> 64 -> 1, tanh hidden, linear output) in BF16 on MFMA."""

    def __init__(self, weights, biases, device="cuda", stream=None):
        in_dim, hidden = weights[0].shape
        self.in_dim, self.hidden = int(in_dim), int(hidden)
        self._host = pack_policy_weights(weights, biases)
        nbytes = lib().pol_workspace_bytes(self.in_dim, self.hidden)
        if nbytes == 0:
            raise FlockError(ENV_EINVAL, last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        check(lib().pol_create_value(self._host.ctypes.data, self.in_dim, self.hidden,
                                     self.workspace.data_ptr(), nbytes, _stream(stream),
                                     ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.pol_destroy(h)
            self.handle = None

    def value(self, obs, out=None, stream=None):
        """V [n] for obs [n, in_dim] (any leading shape is flattened to rows)."""
        rows = obs.reshape(-1, self.in_dim)
        n = rows.shape[0]
        if out is None:
            out = torch.empty(obs.shape[:-1], dtype=torch.float32, device=obs.device)
        _dev_f32(rows, (n, self.in_dim), "obs")
        if not (out.is_contiguous() and out.numel() == n and out.dtype == torch.float32):
            raise ValueError("out must be a contiguous float32 tensor with one value per row")
        check(lib().pol_value(self.handle, _ptr(rows), n, _ptr(out), _stream(stream)))
        return out


def gae(reward, value, gamma, lam, adv=None, ret=None, stream=None):
    """Truncated advantage estimator over [steps, n] rewards and [steps + 1, n] values."""
    steps, n = reward.shape
    if adv is None:
        adv = torch.empty_like(reward)
    if ret is None:
        ret = torch.empty_like(reward)
    _dev_f32(reward, (steps, n), "reward")
    _dev_f32(value, (steps + 1, n), "value")
    _dev_f32(adv, (steps, n), "adv")
    _dev_f32(ret, (steps, n), "ret")
    check(lib().rl_gae(int(steps), int(n), float(gamma), float(lam), _ptr(reward), _ptr(value),
                       _ptr(adv), _ptr(ret), _stream(stream)))
    return adv, ret


def opinion_step(row_ptr, col, weight, op_in, op_out, threshold, strength, lanes=0,
                 stream=None):
    """One step of the opinion-dynamics graph interaction (gr_opinion_step of the C ABI).

    row_ptr int64 [n + 1], col int32 [E], weight float32 [E], op_in/op_out
    float32 [n] (distinct), all CUDA tensors.
    """
    n = op_in.shape[0]
    E = col.shape[0]
    for t, dt, shape, nm in ((row_ptr, torch.int64, (n + 1,), "row_ptr"),
                             (col, torch.int32, (E,), "col"), (weight, torch.float32, (E,), "weight"),
                             (op_in, torch.float32, (n,), "op_in"),
                             (op_out, torch.float32, (n,), "op_out")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()
                and tuple(t.shape) == shape):
            raise TypeError(f"{nm} must be a contiguous CUDA {dt} tensor of shape {shape}")
    check(lib().gr_opinion_step(n, E, _ptr(row_ptr), _ptr(col), _ptr(weight), float(threshold),
                                float(strength), _ptr(op_in), _ptr(op_out), int(lanes),
                                _stream(stream)))
    return op_out


def request_bytes(params: Params) -> int:
    """Arena bytes one serving request with these parameters occupies (0 if invalid)."""
    return int(lib().srv_request_bytes(ctypes.byref(params.c())))


class Server:
    """Continuous-batching episode server (srv_* of the C ABI).

    ``arena_bytes`` of device memory (a torch tensor) is the HBM budget the
    server admits requests against.  Requests share ``policy``.
    """

    QUEUED, RUNNING, FINISHED = 0, 1, 2

    def __init__(self, policy: Policy, arena_bytes: int, max_slots: int = 64, device="cuda",
                 stream=None):
        self.policy = policy
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        h = ctypes.c_void_p()
        check(lib().srv_create(self.arena.data_ptr(), int(arena_bytes), int(max_slots),
                               policy.handle, _stream(self.stream), ctypes.byref(h)))
        self.handle = h
        self.sizes = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.srv_destroy(h)
            self.handle = None

    def submit(self, params: Params, state, steps: int):
        """Queue a request; returns (id, admitted_now).  ``state`` = host (x, y, th, s)."""
        import numpy as np
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in state]
        for a in arrs:
            if a.shape != (params.n_agents,):
                raise ValueError("state arrays must have shape (n_agents,)")
        rid = ctypes.c_int64()
        rc = lib().srv_submit(self.handle, ctypes.byref(params.c()), *[a.ctypes.data for a in arrs],
                              int(steps), ctypes.byref(rid))
        if rc not in (ENV_OK, ENV_EAGAIN):
            check(rc)
        self.sizes[rid.value] = params.n_agents
        return rid.value, rc == ENV_OK

    def tick(self):
        """One serving tick; returns (requests stepped, agents stepped)."""
        n, a = ctypes.c_int32(), ctypes.c_int64()
        check(lib().srv_tick(self.handle, ctypes.byref(n), ctypes.byref(a)))
        return n.value, a.value

    def poll(self, rid: int):
        st, done = ctypes.c_int32(), ctypes.c_int32()
        check(lib().srv_poll(self.handle, int(rid), ctypes.byref(st), ctypes.byref(done)))
        return st.value, done.value

    def result(self, rid: int):
        import numpy as np
        n = self.sizes.pop(rid)
        out = np.zeros(n, np.float64)
        check(lib().srv_result(self.handle, int(rid), out.ctypes.data if n else None, n))
        return out
