"""Pins of the plane-projection oracle (oracle.planes, Section 4, eqs. 11-17).

Each projection is checked for what defines it: the two-dimensional divergence vanishes
in every plane, the dropped component and the wall-normal faces are zero, it is
idempotent, the residual is orthogonal (face-volume inner product) to the subspace,
fields already in the subspace are kept and plane gradients removed; the potentials
vanish on the walls and their curl gives the projection back.
"""
import numpy as np
import pytest

from oracle import planes
from oracle.fv import divergence, gradient, zero_walls
from oracle.grid import Grid


def grids():
    return [Grid.make(6, 5, 4, kind="sine"), Grid.make(5, 4, 6, kind="tanh", ratio=4.0)]


def mdot(g, a, b):
    mu, mv, mw = g.face_volumes()
    return float(np.dot(g.pack(mu, mv, mw) * a, b))


@pytest.mark.parametrize("which", [1, 2, 3])
@pytest.mark.parametrize("gi", [0, 1])
def test_projection_defining_properties(which, gi):
    g = grids()[gi]
    rng = np.random.default_rng(10 * which + gi)
    b = rng.standard_normal(g.nvel())
    p, _ = planes.project_plane(g, b, which)
    u, v, w = g.unpack(p)
    keep = planes.KEEP[which]
    # dropped component and wall-normal faces are zero
    for c, k in zip((u, v, w), keep):
        if not k:
            assert np.all(c == 0.0)
    assert np.all(p[g.wall_mask()] == 0.0)
    # two-dimensional divergence vanishes in every plane (the third component is 0)
    assert np.max(np.abs(divergence(g, p))) < 1e-11 * np.max(np.abs(divergence(g, b)))
    # idempotent
    pp, _ = planes.project_plane(g, p, which)
    assert np.allclose(pp, p, rtol=0, atol=1e-12 * np.abs(p).max())
    # orthogonal: the residual of the kept components is M-orthogonal to the subspace
    a, _ = planes.project_plane(g, rng.standard_normal(g.nvel()), which)
    bk = zero_walls(g, planes._mask(g, b, keep))
    assert abs(mdot(g, bk - p, a)) < 1e-11 * np.sqrt(mdot(g, bk, bk) * mdot(g, a, a))


@pytest.mark.parametrize("which", [1, 2, 3])
def test_subspace_kept_and_gradients_removed(which):
    g = grids()[0]
    rng = np.random.default_rng(40 + which)
    # a curl of a potential vanishing on the walls is in the subspace
    shape = planes.potential(g, np.zeros(g.nvel()), which).shape
    psi = np.zeros(shape)
    psi[tuple(slice(1, -1) if s > 2 else slice(None) for s in shape)] = 0.0
    inner = rng.standard_normal(shape)
    if which == 1:
        inner[:, :, 0] = inner[:, :, -1] = 0.0
        inner[0] = inner[-1] = 0.0
    elif which == 2:
        inner[:, 0] = inner[:, -1] = 0.0
        inner[0] = inner[-1] = 0.0
    else:
        inner[:, :, 0] = inner[:, :, -1] = 0.0
        inner[:, 0] = inner[:, -1] = 0.0
    a = planes.curl_of_potential(g, inner, which)
    assert np.all(a[g.wall_mask()] == 0.0)
    pa, _ = planes.project_plane(g, a, which)
    assert np.allclose(pa, a, rtol=0, atol=1e-12 * np.abs(a).max())
    # a plane gradient (normal component dropped) is removed
    phi = rng.standard_normal((g.nz, g.ny, g.nx))
    gr = planes._mask(g, gradient(g, phi), planes.KEEP[which])
    pg, _ = planes.project_plane(g, gr, which)
    assert np.max(np.abs(pg)) < 1e-11 * np.max(np.abs(gr))


@pytest.mark.parametrize("which", [1, 2, 3])
def test_potential_vanishes_on_walls_and_reproduces_the_projection(which):
    g = grids()[1]
    b = np.random.default_rng(50 + which).standard_normal(g.nvel())
    p, _ = planes.project_plane(g, b, which)
    psi = planes.potential(g, p, which)
    scale = np.abs(psi).max()
    if which == 1:
        walls = [psi[0], psi[-1], psi[:, :, 0], psi[:, :, -1]]
    elif which == 2:
        walls = [psi[0], psi[-1], psi[:, 0], psi[:, -1]]
    else:
        walls = [psi[:, 0], psi[:, -1], psi[:, :, 0], psi[:, :, -1]]
    for wall in walls:
        assert np.max(np.abs(wall)) < 1e-12 * scale
    back = planes.curl_of_potential(g, psi, which)
    assert np.allclose(back, p, rtol=0, atol=1e-11 * np.abs(p).max())


@pytest.mark.parametrize("which", [1, 2, 3])
@pytest.mark.parametrize("gi", [0, 1])
def test_one_plane_sparse_solve_matches_the_dense_projection(which, gi):
    # the single-plane sparse solve (for sampling large grids) against the dense
    # projection and potential on every plane
    g = grids()[gi]
    b = np.random.default_rng(60 + 10 * gi + which).standard_normal(g.nvel())
    p, _ = planes.project_plane(g, b, which)
    u, v, w = g.unpack(p)
    psi = planes.potential(g, p, which)
    n = {1: g.ny, 2: g.nx, 3: g.nz}[which]
    for idx in range(n):
        first, second, ps = planes.project_one_plane(g, b, which, idx)
        if which == 1:
            ref = (u[:, idx, :], w[:, idx, :], psi[:, idx, :])
        elif which == 2:
            ref = (v[:, :, idx], w[:, :, idx], psi[:, :, idx])
        else:
            ref = (u[idx], v[idx], psi[idx])
        for a, r in zip((first, second, ps), ref):
            assert a.shape == r.shape
            assert np.max(np.abs(a - r)) < 1e-12 * max(np.abs(r).max(), 1.0)
