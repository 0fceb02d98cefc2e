"""Stokes-preconditioned (time-stepper) Krylov vectors (Section 3, refs. [35-37]).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper contrasts its SIMPLE-evaluated Krylov vectors with Krylov vectors taken from
time steps whose viscous part is implicit (Stokes preconditioning).  The pieces,
written out plainly:

* the viscous operator Lap_0 (the vector Laplacian of eq. 2 with zero wall values) as a
  sparse matrix per velocity component, the Kronecker sum of three 1D second
  differences: along the component's own axis over its faces (the wall faces hold
  zero), along the other two over cells with the zero wall value reached over a half
  width;
* the viscous step u = (I/dt - Re^-1 Lap_0)^-1 f by a sparse direct solve on the
  interior faces (dt = inf: the Stokes operator -Re^-1 Lap_0);
* the Stokes step P (viscous step of f), and the Stokes-preconditioned Krylov vector
  P (I/dt - Re^-1 Lap_0)^-1 P L_U v.

The Laplacian here is assembled independently of ``fv.laplacian`` (Kronecker products
of 1D matrices against slicing of arrays); the pins compare the two.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .grid import Axis, Grid
from .simple import Projector


def face_second_difference(ax: Axis):
    """1D second difference of a component along its own axis, on the n+1 faces
    (rows of the wall faces 0 and n are zero; their values are zero)."""
    n = ax.n
    A = sp.lil_matrix((n + 1, n + 1))
    for i in range(1, n):
        A[i, i - 1] = 1.0 / (ax.d[i - 1] * ax.dd[i])
        A[i, i] = -(1.0 / ax.d[i - 1] + 1.0 / ax.d[i]) / ax.dd[i]
        A[i, i + 1] = 1.0 / (ax.d[i] * ax.dd[i])
    return A.tocsr()


def cell_second_difference(ax: Axis):
    """1D second difference along an axis on which the component is cell-centred;
    the zero wall value enters through the half-width fluxes at faces 0 and n."""
    n = ax.n
    A = sp.lil_matrix((n, n))
    for j in range(n):
        A[j, j] = -(1.0 / ax.dd[j] + 1.0 / ax.dd[j + 1]) / ax.d[j]
        if j > 0:
            A[j, j - 1] = 1.0 / (ax.dd[j] * ax.d[j])
        if j < n - 1:
            A[j, j + 1] = 1.0 / (ax.dd[j + 1] * ax.d[j])
    return A.tocsr()


def component_laplacian(g: Grid, comp: int):
    """Sparse Lap_0 of one component (0: u, 1: v, 2: w) on its full array, x fastest."""
    mats = []
    for axis_index, ax in enumerate((g.X, g.Y, g.Z)):
        mats.append(face_second_difference(ax) if axis_index == comp else cell_second_difference(ax))
    Ax, Ay, Az = mats
    Ix, Iy, Iz = (sp.identity(m.shape[0], format="csr") for m in mats)
    # flattened index = (k * Ly + j) * Lx + i  ->  kron(z, kron(y, x))
    return (sp.kron(Iz, sp.kron(Iy, Ax)) + sp.kron(Iz, sp.kron(Ay, Ix)) + sp.kron(Az, sp.kron(Iy, Ix))).tocsr()


def laplacian_matrix(g: Grid):
    """Block-diagonal sparse Lap_0 on the packed velocity u|v|w."""
    return sp.block_diag([component_laplacian(g, c) for c in range(3)], format="csr")


def viscous_solve(g: Grid, f, re: float, dt: float):
    """u = (I/dt - Re^-1 Lap_0)^-1 f on the interior faces, zero on the walls."""
    L = laplacian_matrix(g)
    it = np.nonzero(~g.wall_mask())[0]
    rdt = 0.0 if np.isinf(dt) else 1.0 / dt
    H = (rdt * sp.identity(g.nvel(), format="csr") - L / re)[it][:, it].tocsc()
    u = np.zeros(g.nvel())
    u[it] = spla.spsolve(H, np.asarray(f, dtype=np.float64)[it])
    return u


def stokes_step(g: Grid, f, re: float, dt: float):
    """P (I/dt - Re^-1 Lap_0)^-1 f: the viscous step, then the projection."""
    return Projector(g).project(viscous_solve(g, f, re, dt))[0]


def stokes_vector(g: Grid, U, v, re: float, dt: float):
    """The Stokes-preconditioned Krylov vector P (I/dt - Re^-1 Lap_0)^-1 P L_U v."""
    w, _ = Projector(g).krylov_vector(U, v, re)
    return stokes_step(g, w, re, dt)
