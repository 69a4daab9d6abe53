"""Run parameters of the DSMC channel in the library's nondimensional units.

Units: cell size 1, kT/m = 1 by default, so speeds are in units of the
thermal speed sqrt(kT/m) (the appendix's scaling factors, with the lattice
speed of sound matched to the isothermal sound speed of the gas).
"""
from __future__ import annotations

import math
from dataclasses import dataclass


def time_step(kn: float, ny: int, kT: float = 1.0) -> float:
    """min of a quarter cell at the most probable speed and a fifth of the mean collision time."""
    lam = kn * float(ny)
    cbar = math.sqrt(8.0 * kT / math.pi)
    return min(0.25 / math.sqrt(2.0 * kT), 0.2 * lam / cbar)


def hard_sphere_viscosity(kn: float, ny: int, kT: float = 1.0) -> float:
    """Chapman-Enskog kinematic viscosity of hard spheres: (5/16) sqrt(2 pi) 1.016 lambda sqrt(kT/m)."""
    return (5.0 / 16.0) * math.sqrt(2.0 * math.pi) * 1.016 * kn * float(ny) * math.sqrt(kT)


def body_force(kn: float, ny: int, mach: float, kT: float = 1.0) -> float:
    """Acceleration giving a no-slip centreline speed mach * sqrt(kT/m): g = 8 nu U / H^2."""
    return 8.0 * hard_sphere_viscosity(kn, ny, kT) * mach * math.sqrt(kT) / float(ny) ** 2


def bgk_tau(kn: float, ny: int, c_over_cs: float) -> float:
    """Eq. (tau): relaxation time of the BGK lattice for Knudsen number kn on height ny."""
    return math.sqrt(math.pi / 8.0) * c_over_cs * kn * float(ny) + 0.5


@dataclass
class ChannelConfig:
    nx: int
    ny: int
    ppc: int
    kn: float
    mach: float = 0.0
    dt: float | None = None
    body_force_x: float | None = None
    kT_over_m: float = 1.0
    sigcr_max0: float = 6.0
    seed: int = 1
    capacity: int | None = None
    nbar_mode: int = 0
    ar_max_tries: int = 0
    far_capacity: int = 0
    state_bits: int = 64  # 64: FP64 particle state; 32: FP32 storage, FP64 arithmetic

    def resolved(self) -> "ChannelConfig":
        c = ChannelConfig(**self.__dict__)
        if c.dt is None:
            c.dt = time_step(c.kn, c.ny, c.kT_over_m)
        if c.body_force_x is None:
            c.body_force_x = body_force(c.kn, c.ny, c.mach, c.kT_over_m) if c.mach else 0.0
        if c.capacity is None:
            c.capacity = int(c.nx * c.ny * c.ppc * 1.25) + 1024
        return c
