"""MI355X-native DSMC particle step and DSMC<->LBM mapping (arXiv:1512.08042).

The hot path runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/dsmc.h (libdsmc.so); this package only marshals arguments.
"""
from .config import ChannelConfig, bgk_tau, body_force, hard_sphere_viscosity, time_step  # noqa: F401

__all__ = ["ChannelConfig", "bgk_tau", "body_force", "hard_sphere_viscosity", "time_step", "Channel", "lattice",
           "lbm_step", "project_moments"]


def __getattr__(name):
    if name in ("Channel", "lattice", "lbm_step", "project_moments"):
        from . import dsmc

        return getattr(dsmc, name)
    raise AttributeError(name)
