"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module holds no arithmetic of the method: it only draws random numbers
(numpy's PCG64) and lays them out.  Anything method-specific (lattice weights,
equilibria, coefficients) is passed in by the caller.
"""
from __future__ import annotations

import numpy as np


def particles(seed: int, nx: int, ny: int, n: int, vscale: float = 1.0, vmean=(0.0, 0.0, 0.0)):
    """n particles uniform over [0,nx) x [0,ny), Gaussian velocities."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, nx, n)
    y = rng.uniform(0.0, ny, n)
    v = rng.normal(0.0, vscale, (3, n))
    return x, y, v[0] + vmean[0], v[1] + vmean[1], v[2] + vmean[2]


def particles_per_cell(seed: int, nx: int, ny: int, counts, vscale: float = 1.0):
    """counts[c] particles uniform inside cell c, shuffled slot order."""
    rng = np.random.default_rng(seed)
    counts = np.asarray(counts, dtype=np.int64)
    cid = np.repeat(np.arange(nx * ny), counts)
    rng.shuffle(cid)
    x = (cid % nx) + rng.uniform(0.0, 1.0, cid.size)
    y = (cid // nx) + rng.uniform(0.0, 1.0, cid.size)
    v = rng.normal(0.0, vscale, (3, cid.size))
    return x, y, v[0], v[1], v[2]


def populations(seed: int, base, ncells: int, eps: float):
    """f[a][c] = base[a] * (1 + eps * U(-1, 1)), independent per entry."""
    rng = np.random.default_rng(seed)
    base = np.asarray(base, dtype=np.float64)
    return base[:, None] * (1.0 + eps * rng.uniform(-1.0, 1.0, (base.size, ncells)))


def moment_sums(seed: int, ncells: int, scale: float = 1.0):
    """An [11][ncells] array of positive counts and arbitrary sums (for projection parity)."""
    rng = np.random.default_rng(seed)
    m = rng.normal(0.0, scale, (11, ncells))
    m[0] = rng.uniform(50.0, 150.0, ncells)
    return m


def strip_cells(nx: int, ny: int, width: int):
    """Cell ids of the strip 0 <= ix < width over all rows."""
    ix = np.arange(width)
    iy = np.arange(ny)
    return (iy[:, None] * nx + ix[None, :]).ravel().astype(np.int32)


def replica_params(seed: int, n: int, ny_range=(32, 512), ppc_range=(20, 200), kn_range=(0.01, 1.0)):
    """n independent channel replicas of one cell across x: ny and ppc uniform
    integers over the closed ranges, Kn log-uniform over kn_range, seeds
    1000 + index."""
    rng = np.random.default_rng(seed)
    ny = rng.integers(ny_range[0], ny_range[1] + 1, n)
    ppc = rng.integers(ppc_range[0], ppc_range[1] + 1, n)
    kn = np.exp(rng.uniform(np.log(kn_range[0]), np.log(kn_range[1]), n))
    return [dict(nx=1, ny=int(a), ppc=int(b), kn=float(c), seed=1000 + i)
            for i, (a, b, c) in enumerate(zip(ny, ppc, kn))]
