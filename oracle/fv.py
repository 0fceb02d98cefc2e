"""Staggered finite-volume operators of the lid-driven cube (Sections 2-3).

The paper defers the discretization to its ref. [31]; this oracle uses the
marker-and-cell reading stated here, all terms per unit volume:

* Divergence (eq. 1) at cell (i,j,k):
  (u[i+1]-u[i])/dX[i] + (v[j+1]-v[j])/dY[j] + (w[k+1]-w[k])/dZ[k].
* Gradient on interior faces: (p[i]-p[i-1])/ddX[i]; zero on wall faces.
* Laplacian (eq. 2) of a component along its own (normal) axis uses the faces
  i-1, i, i+1 (wall faces hold zero).  Along a tangential axis the fluxes sit on
  the cell faces; at a wall the flux is (first value - wall value)/half width,
  with the wall value of eqs. 3-4 (cos a for u and sin a for v at z = 1, zero
  elsewhere).  Corner values never enter (Section 5.1).
* Convection is conservative, C(a, b) = div(a (x) b), with a the advecting and
  b the advected field: centred averages at cell centres for the normal flux,
  and for the tangential fluxes the product, on cell edges, of the advecting
  component interpolated along the momentum axis and the advected component
  interpolated along the flux axis; edge fluxes on a wall vanish because the
  wall-normal velocity does.
* Momentum residual R(U) = Re^-1 Lap_g U - C(U, U) (eq. 2 at steady state,
  pressure left to the projection), and its exact Jacobian
  L_U v = Re^-1 Lap_0 v - C(U, v) - C(v, U), the right side of eq. 10 (the
  linearized momentum of eq. 6).  C is bilinear, so
  R(U + e v) = R(U) + e L_U v - e^2 C(v, v) exactly.

Velocity arguments are packed vectors u|v|w (see ``grid.Grid.pack``); outputs
are packed the same way with zero on every wall-normal face.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid


def _b(a, axis):
    """Reshape a 1D metric array to broadcast along array axis (0=z, 1=y, 2=x)."""
    shape = [1, 1, 1]
    shape[axis] = -1
    return np.asarray(a).reshape(shape)


def _sl(axis, s):
    idx = [slice(None)] * 3
    idx[axis] = s
    return tuple(idx)


def _axis(g: Grid, axis):
    return (g.Z, g.Y, g.X)[axis]


def zero_walls(g: Grid, vec):
    """Return a copy of a packed velocity with every wall-normal face set to 0."""
    out = np.array(vec, dtype=np.float64, copy=True)
    out[g.wall_mask()] = 0.0
    return out


# ----------------------------------------------------------------- div / grad
def divergence(g: Grid, vec):
    """Cell-centred divergence of a packed velocity (eq. 1)."""
    u, v, w = g.unpack(vec)
    return (np.diff(u, axis=2) / _b(g.X.d, 2)
            + np.diff(v, axis=1) / _b(g.Y.d, 1)
            + np.diff(w, axis=0) / _b(g.Z.d, 0))


def gradient(g: Grid, p):
    """Face gradient of a cell field, zero on wall faces."""
    su, sv, sw, _ = g.shapes()
    gu = np.zeros(su); gv = np.zeros(sv); gw = np.zeros(sw)
    gu[:, :, 1:-1] = np.diff(p, axis=2) / _b(g.X.dd[1:-1], 2)
    gv[:, 1:-1, :] = np.diff(p, axis=1) / _b(g.Y.dd[1:-1], 1)
    gw[1:-1] = np.diff(p, axis=0) / _b(g.Z.dd[1:-1], 0)
    return g.pack(gu, gv, gw)


# ------------------------------------------------------------------ Laplacian
def _lap_normal(f, ax, axis):
    """Second difference of a face component along its own axis (faces 1..n-1)."""
    n = ax.n
    grad = np.diff(f, axis=axis) / _b(ax.d, axis)            # at cell centres
    out = np.zeros_like(f)
    out[_sl(axis, slice(1, n))] = np.diff(grad, axis=axis) / _b(ax.dd[1:n], axis)
    return out


def _lap_tangential(f, ax, axis, g_lo, g_hi):
    """Second difference along an axis on which the component is cell-centred;
    wall values g_lo (at x=0) and g_hi (at x=1) enter through half-width fluxes."""
    n = ax.n
    first = f[_sl(axis, slice(0, 1))]
    last = f[_sl(axis, slice(n - 1, n))]
    flux = np.concatenate([
        (first - g_lo) / ax.dd[0],
        np.diff(f, axis=axis) / _b(ax.dd[1:n], axis),
        (g_hi - last) / ax.dd[n],
    ], axis=axis)
    return np.diff(flux, axis=axis) / _b(ax.d, axis)


def laplacian(g: Grid, vec, lid=None):
    """Vector Laplacian of a packed velocity.

    ``lid`` is None for the homogeneous conditions, or (u_top, v_top) for the
    moving lid at z = 1 (eq. 4, u = cos a, v = sin a).
    """
    u, v, w = g.unpack(vec)
    ut, vt = (0.0, 0.0) if lid is None else lid
    lu = (_lap_normal(u, g.X, 2) + _lap_tangential(u, g.Y, 1, 0.0, 0.0)
          + _lap_tangential(u, g.Z, 0, 0.0, ut))
    lv = (_lap_normal(v, g.Y, 1) + _lap_tangential(v, g.X, 2, 0.0, 0.0)
          + _lap_tangential(v, g.Z, 0, 0.0, vt))
    lw = (_lap_normal(w, g.Z, 0) + _lap_tangential(w, g.X, 2, 0.0, 0.0)
          + _lap_tangential(w, g.Y, 1, 0.0, 0.0))
    return zero_walls(g, g.pack(lu, lv, lw))


# ----------------------------------------------------------------- convection
def _to_centre(f, axis):
    """Average of the two faces of each cell along ``axis``."""
    return 0.5 * (f[_sl(axis, slice(0, -1))] + f[_sl(axis, slice(1, None))])


def _to_faces(f, ax, axis):
    """Interpolate a cell-centred quantity (n entries along ``axis``) to the n+1
    faces: interior face i gets (1-th[i]) f[i-1] + th[i] f[i]; the two wall
    entries are set to 0 (every flux that uses them vanishes)."""
    n = ax.n
    shape = list(f.shape)
    shape[axis] = n + 1
    out = np.zeros(shape)
    th = _b(ax.th[1:n], axis)
    out[_sl(axis, slice(1, n))] = ((1.0 - th) * f[_sl(axis, slice(0, n - 1))]
                                   + th * f[_sl(axis, slice(1, n))])
    return out


def convection(g: Grid, a_vec, b_vec):
    """Conservative convection C(a, b) = div(a (x) b) on the staggered grid."""
    X, Y, Z = g.X, g.Y, g.Z
    au, av, aw = g.unpack(a_vec)
    bu, bv, bw = g.unpack(b_vec)
    su, sv, sw, _ = g.shapes()

    # u-momentum, unknown at (xf[i], yc[j], zc[k])
    cu = np.zeros(su)
    xc = _to_centre(au, 2) * _to_centre(bu, 2)                     # at cell centres
    cu[:, :, 1:-1] = np.diff(xc, axis=2) / _b(X.dd[1:-1], 2)
    e = _to_faces(av, X, 2) * _to_faces(bu, Y, 1)                 # edges (xf, yf, zc)
    e[:, 0, :] = 0.0; e[:, -1, :] = 0.0
    cu += np.diff(e, axis=1) / _b(Y.d, 1)
    e = _to_faces(aw, X, 2) * _to_faces(bu, Z, 0)                 # edges (xf, yc, zf)
    e[0] = 0.0; e[-1] = 0.0
    cu += np.diff(e, axis=0) / _b(Z.d, 0)

    # v-momentum, unknown at (xc[i], yf[j], zc[k])
    cv = np.zeros(sv)
    e = _to_faces(au, Y, 1) * _to_faces(bv, X, 2)                 # edges (xf, yf, zc)
    e[:, :, 0] = 0.0; e[:, :, -1] = 0.0
    cv += np.diff(e, axis=2) / _b(X.d, 2)
    yc = _to_centre(av, 1) * _to_centre(bv, 1)
    cv[:, 1:-1, :] += np.diff(yc, axis=1) / _b(Y.dd[1:-1], 1)
    e = _to_faces(aw, Y, 1) * _to_faces(bv, Z, 0)                 # edges (xc, yf, zf)
    e[0] = 0.0; e[-1] = 0.0
    cv += np.diff(e, axis=0) / _b(Z.d, 0)

    # w-momentum, unknown at (xc[i], yc[j], zf[k])
    cw = np.zeros(sw)
    e = _to_faces(au, Z, 0) * _to_faces(bw, X, 2)                 # edges (xf, yc, zf)
    e[:, :, 0] = 0.0; e[:, :, -1] = 0.0
    cw += np.diff(e, axis=2) / _b(X.d, 2)
    e = _to_faces(av, Z, 0) * _to_faces(bw, Y, 1)                 # edges (xc, yf, zf)
    e[:, 0, :] = 0.0; e[:, -1, :] = 0.0
    cw += np.diff(e, axis=1) / _b(Y.d, 1)
    zc = _to_centre(aw, 0) * _to_centre(bw, 0)
    cw[1:-1] += np.diff(zc, axis=0) / _b(Z.dd[1:-1], 0)

    return zero_walls(g, g.pack(cu, cv, cw))


# ------------------------------------------------- residual and its Jacobian
def lid_values(alpha):
    """Lid velocity (u, v) at z = 1 for direction angle alpha (eq. 4); None gives
    a resting lid (homogeneous walls, used for manufactured solutions)."""
    if alpha is None:
        return None
    return (np.cos(alpha), np.sin(alpha))


def residual(g: Grid, U, re: float, alpha):
    """Momentum residual R(U) = Re^-1 Lap_g U - C(U, U) with the lid of eq. 4."""
    U = zero_walls(g, U)
    return laplacian(g, U, lid_values(alpha)) / re - convection(g, U, U)


def jacobian_apply(g: Grid, U, v, re: float):
    """L_U v = Re^-1 Lap_0 v - C(U, v) - C(v, U): right side of eq. 10."""
    U = zero_walls(g, U)
    v = zero_walls(g, v)
    return laplacian(g, v) / re - convection(g, U, v) - convection(g, v, U)
