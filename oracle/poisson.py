"""Exact Neumann pressure-correction Poisson solve (Section 3, step 1).

The discrete operator is A = D G, the divergence of the face gradient with the
gradient held at zero on the walls (the Neumann condition of step 1).  On the
tensor-product grid A is the Kronecker sum of three 1D operators
A_x = M_x^-1 K_x with M_x = diag(dX) and K_x the symmetric tridiagonal matrix of
couplings 1/ddX on interior faces.  Following the full tensor-product
factorization (TPF) the paper uses on its finest grids, each 1D generalized
symmetric eigenproblem K s = lam M s is solved once (S^T M S = I), the right
side is transformed along x, y, z with S^T M, divided by lam_x + lam_y + lam_z,
and transformed back with S.  The constant mode (lam = 0 on every axis) is set to
zero, which fixes sum_c V_c phi_c = 0.  The result is exact to rounding.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .grid import Axis, Grid


def axis_operator(ax: Axis):
    """(K, M) of the 1D Neumann operator A = M^-1 K on one axis."""
    n = ax.n
    K = np.zeros((n, n))
    for i in range(1, n):           # interior face i couples cells i-1 and i
        c = 1.0 / ax.dd[i]
        K[i - 1, i - 1] -= c
        K[i, i] -= c
        K[i - 1, i] += c
        K[i, i - 1] += c
    M = np.diag(ax.d)
    return K, M


def axis_modes(ax: Axis):
    """Generalized eigenpairs (lam ascending, S with S^T M S = I) of one axis."""
    K, M = axis_operator(ax)
    lam, S = scipy.linalg.eigh(K, M)
    return lam, S, M


def _along(mat, f, axis):
    """Apply matrix ``mat`` to every line of ``f`` along ``axis``."""
    return np.moveaxis(np.tensordot(mat, np.moveaxis(f, axis, 0), axes=(1, 0)), 0, axis)


class PoissonFD:
    """Fast-diagonalization solver of (D G) phi = r with sum V phi = 0."""

    def __init__(self, g: Grid):
        self.g = g
        self.modes = [axis_modes(ax) for ax in (g.Z, g.Y, g.X)]   # array axes 0,1,2
        lz, ly, lx = (m[0] for m in self.modes)
        den = lz[:, None, None] + ly[None, :, None] + lx[None, None, :]
        # the single zero mode: lam = 0 on each axis, the largest (last) eigenvalue
        zero = np.zeros(den.shape, bool)
        zero[-1, -1, -1] = True
        self.inv = np.where(zero, 0.0, 1.0 / np.where(zero, 1.0, den))

    def solve(self, r):
        r = np.asarray(r, dtype=np.float64)
        c = r
        for axis, (_, S, M) in enumerate(self.modes):
            c = _along(S.T @ M, c, axis)
        c = c * self.inv
        for axis, (_, S, _) in enumerate(self.modes):
            c = _along(S, c, axis)
        return c


def apply_DG(g: Grid, phi):
    """Direct evaluation of (D G) phi, for checks."""
    from .fv import divergence, gradient
    return divergence(g, gradient(g, phi))
