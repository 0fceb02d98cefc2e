"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only draws pseudo-random
numbers and lays them out in the staggered field shapes.  The generator is
SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used in counter mode: element ``i`` of stream
``seed`` is ``mix(seed + (i + 1) * GOLDEN)``.  A uniform double in [0, 1) is the
top 53 bits times 2**-53; it is mapped to [-1, 1) by ``2*u - 1``.

Field layout (x fastest, C order), for Nx x Ny x Nz finite volumes:

* ``u``: (Nz, Ny, Nx+1)  -- x-faces; faces i = 0 and i = Nx are walls
* ``v``: (Nz, Ny+1, Nx)  -- y-faces; faces j = 0 and j = Ny are walls
* ``w``: (Nz+1, Ny, Nx)  -- z-faces; faces k = 0 and k = Nz are walls
* ``p``: (Nz, Ny, Nx)    -- cell centres

A packed velocity vector is ``u | v | w`` flattened in that order.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Return ``n`` SplitMix64 outputs of stream ``seed`` starting at counter ``offset``."""
    with np.errstate(over="ignore"):
        ctr = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + ctr * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """``n`` doubles uniform in [-1, 1) from stream ``seed``."""
    z = splitmix64(seed, n, offset)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


def shapes(nx: int, ny: int, nz: int):
    """Shapes of (u, v, w, p) for an Nx x Ny x Nz grid."""
    return ((nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx), (nz, ny, nx))


def vel_size(nx: int, ny: int, nz: int) -> int:
    su, sv, sw, _ = shapes(nx, ny, nz)
    return int(np.prod(su) + np.prod(sv) + np.prod(sw))


def interior_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    """Boolean packed-velocity mask: True on every face that is not a wall face."""
    su, sv, sw, _ = shapes(nx, ny, nz)
    mu = np.ones(su, bool); mu[:, :, 0] = False; mu[:, :, -1] = False
    mv = np.ones(sv, bool); mv[:, 0, :] = False; mv[:, -1, :] = False
    mw = np.ones(sw, bool); mw[0] = False; mw[-1] = False
    return np.concatenate([mu.ravel(), mv.ravel(), mw.ravel()])


def random_velocity(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    """Packed velocity, uniform [-1, 1) on interior faces, exactly 0 on wall faces."""
    n = vel_size(nx, ny, nz)
    x = uniform_pm1(seed, n)
    x[~interior_mask(nx, ny, nz)] = 0.0
    return x


def random_cells(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    """Cell field (Nz, Ny, Nx) uniform in [-1, 1)."""
    return uniform_pm1(seed, nx * ny * nz).reshape(nz, ny, nx)
