"""Stretched staggered grid of the unit cube (Section 3, eq. 5).

Each axis has faces x_f[0..N] with x_f[0] = 0, x_f[N] = 1 (the N+1 points of
Section 3 bound N finite volumes).  Metrics, 0-based:

* ``d[i]  = x_f[i+1] - x_f[i]``            cell width, i = 0..N-1
* ``c[i]  = (x_f[i] + x_f[i+1]) / 2``      cell centre
* ``dd[i] = c[i] - c[i-1]``                centre-to-centre distance across face i,
  i = 1..N-1; at the walls the half widths ``dd[0] = d[0]/2``, ``dd[N] = d[N-1]/2``
* ``th[i] = d[i-1] / (2 dd[i])``            weight that interpolates a cell
  quantity to face i: ``(1 - th) a[i-1] + th a[i]``
"""
from __future__ import annotations

import numpy as np

SINE_AMPLITUDE = 0.0975  # Section 3, eq. 5


def faces(n: int, kind: str = "uniform", ratio: float = 10.0) -> np.ndarray:
    """Face coordinates of one axis.

    ``uniform``: x_i = i/N.
    ``sine``:    x_i -> x_i - 0.0975 sin(2 pi x_i)   (Section 3, eq. 5).
    ``tanh``:    x = (1 + tanh(b (2 xi - 1)) / tanh b) / 2 with cosh^2 b = ratio, so
                 that the continuous centre/wall spacing ratio equals ``ratio``.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    xi = np.arange(n + 1, dtype=np.float64) / n
    if kind == "uniform":
        x = xi.copy()
    elif kind == "sine":
        x = xi - SINE_AMPLITUDE * np.sin(2.0 * np.pi * xi)
    elif kind == "tanh":
        if ratio <= 1.0:
            raise ValueError("tanh ratio must exceed 1")
        b = np.arccosh(np.sqrt(ratio))
        x = 0.5 * (1.0 + np.tanh(b * (2.0 * xi - 1.0)) / np.tanh(b))
    else:
        raise ValueError(f"unknown stretching {kind!r}")
    x[0] = 0.0
    x[-1] = 1.0
    if np.any(np.diff(x) <= 0):
        raise ValueError("faces must increase strictly")
    return x


class Axis:
    """Metrics of one axis built from its faces."""

    def __init__(self, xf):
        xf = np.asarray(xf, dtype=np.float64)
        n = xf.size - 1
        if n < 1 or np.any(np.diff(xf) <= 0):
            raise ValueError("faces must increase strictly")
        self.n = n
        self.xf = xf
        self.d = np.diff(xf)
        self.c = 0.5 * (xf[:-1] + xf[1:])
        dd = np.empty(n + 1)
        dd[0] = 0.5 * self.d[0]
        dd[n] = 0.5 * self.d[-1]
        dd[1:n] = np.diff(self.c)
        self.dd = dd
        th = np.full(n + 1, 0.5)
        th[1:n] = self.d[:-1] / (2.0 * dd[1:n])
        self.th = th


class Grid:
    """Tensor-product grid; arrays are indexed [k, j, i] (z, y, x), x fastest."""

    def __init__(self, xf, yf, zf):
        self.X = Axis(xf)
        self.Y = Axis(yf)
        self.Z = Axis(zf)

    @classmethod
    def make(cls, nx: int, ny: int | None = None, nz: int | None = None,
             kind: str = "uniform", ratio: float = 10.0) -> "Grid":
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        return cls(faces(nx, kind, ratio), faces(ny, kind, ratio), faces(nz, kind, ratio))

    @property
    def nx(self):
        return self.X.n

    @property
    def ny(self):
        return self.Y.n

    @property
    def nz(self):
        return self.Z.n

    def shapes(self):
        nx, ny, nz = self.nx, self.ny, self.nz
        return ((nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx), (nz, ny, nx))

    def nvel(self) -> int:
        return int(sum(np.prod(s) for s in self.shapes()[:3]))

    def unpack(self, vec):
        su, sv, sw, _ = self.shapes()
        a = int(np.prod(su))
        b = a + int(np.prod(sv))
        vec = np.asarray(vec)
        return vec[:a].reshape(su), vec[a:b].reshape(sv), vec[b:].reshape(sw)

    @staticmethod
    def pack(u, v, w):
        return np.concatenate([np.ravel(u), np.ravel(v), np.ravel(w)])

    def volumes(self):
        """Cell volumes V[k, j, i]."""
        return (self.Z.d[:, None, None] * self.Y.d[None, :, None] * self.X.d[None, None, :])

    def face_volumes(self):
        """Control volumes of the u, v, w unknowns (dd of the normal axis times the
        two tangential cell widths)."""
        X, Y, Z = self.X, self.Y, self.Z
        mu = Z.d[:, None, None] * Y.d[None, :, None] * X.dd[None, None, :]
        mv = Z.d[:, None, None] * Y.dd[None, :, None] * X.d[None, None, :]
        mw = Z.dd[:, None, None] * Y.d[None, :, None] * X.d[None, None, :]
        return mu, mv, mw

    def wall_mask(self):
        """Packed boolean mask, True on the wall-normal faces (held at zero)."""
        su, sv, sw, _ = self.shapes()
        mu = np.zeros(su, bool); mu[:, :, 0] = True; mu[:, :, -1] = True
        mv = np.zeros(sv, bool); mv[:, 0, :] = True; mv[:, -1, :] = True
        mw = np.zeros(sw, bool); mw[0] = True; mw[-1] = True
        return self.pack(mu, mv, mw)
