"""Divergence-free projections onto coordinate planes and their vector potentials
(test infrastructure: only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline
leg use this package).

Section 4, eqs. 11-17.  For a velocity field v = (u, v, w):

* v1 = (u1, 0, w1): the orthogonal projection of (u, 0, w) onto the fields with only x
  and z components whose two-dimensional divergence du/dx + dw/dz vanishes in every
  plane y = const (eq. 12) and whose wall-normal components vanish on the walls;
* v2 = (0, v2, w2): the same for (0, v, w) and the planes x = const (eq. 13);
* v3 = (u3, v3, 0): the same for (u, v, 0) and the planes z = const (eq. 14);
* each projection is the curl of a vector potential with one non-zero component
  (eqs. 15-17): v1 = rot(0, Psi_y, 0), v2 = rot(Psi_x, 0, 0), v3 = rot(0, 0, Psi_z).

Discretely, on the staggered grid: the projection is orthogonal in the face-volume
(M-weighted) inner product, so it is b - G2 phi with (D2 G2) phi = D2 b, where D2 and
G2 are the divergence and gradient of the 3D operators with the third component left
out (plane by plane, one Neumann problem per plane).  The potentials live on the cell
edges normal to the planes and vanish on the walls:

* Psi_y at (x-face i, z-face k) of every y-cell: u1 = -dPsi_y/dz, w1 = dPsi_y/dx, built
  from Psi_y(0, k) = 0 by Psi_y(i+1, k) = Psi_y(i, k) + dx_i w1(i, k);
* Psi_x at (y-face j, z-face k) of every x-cell: v2 = dPsi_x/dz, w2 = -dPsi_x/dy, from
  Psi_x(j+1, k) = Psi_x(j, k) - dy_j w2(j, k);
* Psi_z at (x-face i, y-face j) of every z-cell: u3 = dPsi_z/dy, v3 = -dPsi_z/dx, from
  Psi_z(i+1, j) = Psi_z(i, j) - dx_i v3(i, j).

Each plane's Neumann problem is solved densely (minimum-norm least squares, which fixes
the per-plane constant); meant for grids up to a few dozen cells per side.  For sampling
at large sizes, project_one_plane solves a single plane by itself: the same plane operator
assembled explicitly as the sum of the two one-dimensional Neumann operators D_a G_a of its
axes (a sparse matrix), one unknown fixed to zero (the plane gradient does not see the
constant), a sparse direct solve.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fv import divergence, gradient, zero_walls
from .grid import Grid

# which packed components each projection keeps, and the plane axis (0 x, 1 y, 2 z)
KEEP = {1: (True, False, True), 2: (False, True, True), 3: (True, True, False)}
NORMAL = {1: 1, 2: 0, 3: 2}


def _mask(g: Grid, vec, keep):
    u, v, w = (np.array(c, dtype=np.float64) for c in g.unpack(vec))
    for c, k in zip((u, v, w), keep):
        if not k:
            c[...] = 0.0
    return g.pack(u, v, w)


def project_plane(g: Grid, vec, which):
    """The projection v_which (1, 2 or 3) of a packed velocity and its plane pressure."""
    keep, axis = KEEP[which], NORMAL[which]
    b = zero_walls(g, _mask(g, vec, keep))  # wall-normal faces are not unknowns
    ncell = g.nx * g.ny * g.nz
    shape = (g.nz, g.ny, g.nx)

    def op(phi):  # (D2 G2) phi, plane by plane
        return divergence(g, _mask(g, gradient(g, phi.reshape(shape)), keep)).ravel()

    rhs = divergence(g, b).ravel()
    # dense operator of each plane (no coupling across planes: the normal component of
    # the gradient is dropped)
    idx = np.arange(ncell).reshape(shape)
    phi = np.zeros(ncell)
    planes = [np.take(idx, p, axis=2 - axis).ravel() for p in range(shape[2 - axis])]
    for cells in planes:
        A = np.empty((cells.size, cells.size))
        for col, c in enumerate(cells):
            e = np.zeros(ncell)
            e[c] = 1.0
            A[:, col] = op(e)[cells]
        phi[cells] = np.linalg.lstsq(A, rhs[cells], rcond=None)[0]
    out = b - _mask(g, gradient(g, phi.reshape(shape)), keep)
    return out, phi.reshape(shape)


def potential(g: Grid, vec_proj, which):
    """The vector potential of a projection (eqs. 15-17), zero on the walls."""
    u, v, w = g.unpack(vec_proj)
    X, Y = g.X, g.Y
    if which == 1:  # Psi_y[k, j, i], i = 0..nx, k = 0..nz
        psi = np.zeros((g.nz + 1, g.ny, g.nx + 1))
        for i in range(g.nx):
            psi[:, :, i + 1] = psi[:, :, i] + X.d[i] * w[:, :, i]
        return psi
    if which == 2:  # Psi_x[k, j, i], j = 0..ny, k = 0..nz
        psi = np.zeros((g.nz + 1, g.ny + 1, g.nx))
        for j in range(g.ny):
            psi[:, j + 1, :] = psi[:, j, :] - Y.d[j] * w[:, j, :]
        return psi
    psi = np.zeros((g.nz, g.ny + 1, g.nx + 1))  # Psi_z[k, j, i], i = 0..nx, j = 0..ny
    for i in range(g.nx):
        psi[:, :, i + 1] = psi[:, :, i] - X.d[i] * v[:, :, i]
    return psi


def curl_of_potential(g: Grid, psi, which):
    """The packed velocity rot(Psi) of a potential from `potential` (the discrete
    eqs. 15-17; components outside the plane are zero)."""
    su, sv, sw, _ = g.shapes()
    u, v, w = np.zeros(su), np.zeros(sv), np.zeros(sw)
    X, Y, Z = g.X, g.Y, g.Z
    if which == 1:
        u[:] = -np.diff(psi, axis=0) / Z.d[:, None, None]
        w[:] = np.diff(psi, axis=2) / X.d[None, None, :]
    elif which == 2:
        v[:] = np.diff(psi, axis=0) / Z.d[:, None, None]
        w[:] = -np.diff(psi, axis=1) / Y.d[None, :, None]
    else:
        u[:] = np.diff(psi, axis=1) / Y.d[None, :, None]
        v[:] = -np.diff(psi, axis=2) / X.d[None, None, :]
    return g.pack(u, v, w)


# ---------------------------------------------------------------- one plane, sparse
def _neumann_1d(ax):
    """D_a G_a along one axis on cell values: face gradients (phi_f - phi_(f-1)) / dd_f on
    the interior faces, zero through the walls, then the cell differences over d_i."""
    n = ax.n
    f = np.arange(1, n)
    G = sp.csr_matrix((np.concatenate([-1.0 / ax.dd[f], 1.0 / ax.dd[f]]),
                       (np.concatenate([f, f]), np.concatenate([f - 1, f]))), shape=(n + 1, n))
    i = np.arange(n)
    D = sp.csr_matrix((np.concatenate([-1.0 / ax.d, 1.0 / ax.d]),
                       (np.concatenate([i, i]), np.concatenate([i, i + 1]))), shape=(n, n + 1))
    return (D @ G).tocsr()


def project_one_plane(g: Grid, vec, which, index):
    """One plane of projection `which`: the plane normal to the family's axis at cell
    index `index`.  Returns (first, second, psi): the two kept components on that plane
    as 2D arrays (slices of the packed components at the plane, in their natural index
    order: which 1: u[:, index, :], w[:, index, :]; which 2: v[:, :, index], w[:, :, index];
    which 3: u[index], v[index]) and the potential's slice at the plane."""
    keep, axis = KEEP[which], NORMAL[which]
    b = zero_walls(g, _mask(g, vec, keep))
    bu, bv, bw = g.unpack(b)
    rhs3 = divergence(g, b)
    X, Y, Z = g.X, g.Y, g.Z
    if which == 1:  # plane y = index: unknowns phi[k, i]
        slow, fast, rhs = Z, X, rhs3[:, index, :]
    elif which == 2:  # plane x = index: phi[k, j]
        slow, fast, rhs = Z, Y, rhs3[:, :, index]
    else:  # plane z = index: phi[j, i]
        slow, fast, rhs = Y, X, rhs3[index]
    A = (sp.kron(sp.identity(slow.n), _neumann_1d(fast)) + sp.kron(_neumann_1d(slow), sp.identity(fast.n))).tolil()
    r = rhs.ravel().copy()
    A[0, :] = 0.0
    A[0, 0] = 1.0
    r[0] = 0.0
    phi = spla.spsolve(A.tocsc(), r).reshape(slow.n, fast.n)
    # the two kept components minus the plane gradient, zero on the walls
    gf = np.zeros((slow.n, fast.n + 1))
    gf[:, 1:-1] = np.diff(phi, axis=1) / fast.dd[1:-1][None, :]
    gs = np.zeros((slow.n + 1, fast.n))
    gs[1:-1, :] = np.diff(phi, axis=0) / slow.dd[1:-1][:, None]
    if which == 1:
        first, second = bu[:, index, :] - gf, bw[:, index, :] - gs  # u (k, i), w (k, i)
        psi = np.zeros((g.nz + 1, g.nx + 1))  # Psi_y[k, i]
        for i in range(g.nx):
            psi[:, i + 1] = psi[:, i] + X.d[i] * second[:, i]
    elif which == 2:
        first, second = bv[:, :, index] - gf, bw[:, :, index] - gs  # v (k, j), w (k, j)
        psi = np.zeros((g.nz + 1, g.ny + 1))  # Psi_x[k, j]
        for j in range(g.ny):
            psi[:, j + 1] = psi[:, j] - Y.d[j] * second[:, j]
    else:
        first, second = bu[index] - gf, bv[index] - gs  # u (j, i), v (j, i)
        psi = np.zeros((g.ny + 1, g.nx + 1))  # Psi_z[j, i]
        for i in range(g.nx):
            psi[:, i + 1] = psi[:, i] - X.d[i] * second[:, i]
    return first, second, psi
