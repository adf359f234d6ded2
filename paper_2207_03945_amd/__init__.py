"""MI355X (gfx950) flock-environment step library for arXiv:2207.03945.

The step (cell-list hash, neighbour sweep with sector-binned view, proximity
reward and collision penalty, steering and periodic integration) runs in the
HIP kernels of ``libflockenv.so`` behind the C ABI of ``include/flockenv.h``.
``flockenv`` is its ctypes binding.
"""
from .flockenv import (  # noqa: F401
    ENV_FLAG_COUNTS, ENV_FLAG_SPEED_OBS, ENV_FLAG_TAG, Batch, Critic, Env, FlockError, Params, Policy, Server,
    gae, lib, opinion_step, request_bytes, workspace_bytes,
)
