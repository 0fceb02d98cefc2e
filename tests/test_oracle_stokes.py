"""Pins of the oracle's Stokes-preconditioned vectors (oracle/stokes.py).

* The Kronecker-sum viscous operator equals the oracle's stencil Laplacian (fv.laplacian,
  itself pinned by closed forms and the O(h^2) manufactured solution) on random fields
  of uniform, stretched and irregular grids: two independent constructions.
* On a uniform grid the 1D factors have the textbook spectra: -4/h^2 sin^2(m pi / 2n),
  m = 1..n-1 for the face operator (Dirichlet on both walls), m = 1..n for the
  cell-centred one (wall value reached over a half width, i.e. a mirrored ghost).
* The viscous solve satisfies its equation with the stencil Laplacian to rounding.
* The Stokes step is symmetric and positive definite in the face-volume inner product on
  the divergence-free space, maps into it, and tends to dt times the identity there as
  dt -> 0.
"""
import numpy as np
import pytest

import synth
from oracle import fv, simple, stokes
from oracle.grid import Grid


def asym_grid(dims, seed):
    rng = np.random.default_rng(seed)
    fs = []
    for n in dims:
        f = np.concatenate([[0.0], np.cumsum(0.5 + rng.random(n))])
        fs.append(f / f[-1])
    return Grid(*fs)


GRIDS = [Grid.make(6, 5, 4, kind="uniform"), Grid.make(7, 6, 8, kind="tanh"), Grid.make(5, 8, 6, kind="sine"),
         asym_grid((6, 7, 5), 3)]


@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_kronecker_laplacian_equals_stencil(gi):
    g = GRIDS[gi]
    v = synth.random_velocity(g.nx, g.ny, g.nz, 61)
    L = stokes.laplacian_matrix(g)
    it = ~g.wall_mask()
    ref = fv.laplacian(g, v)
    got = L @ v
    assert np.max(np.abs(got[it] - ref[it])) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [4, 7, 12])
def test_uniform_factor_spectra(n):
    g = Grid.make(n, kind="uniform")
    h = 1.0 / n
    F = stokes.face_second_difference(g.X).toarray()[1:n, 1:n]
    Cc = stokes.cell_second_difference(g.X).toarray()
    lf = np.sort(np.linalg.eigvals(F).real)
    lc = np.sort(np.linalg.eigvals(Cc).real)
    ef = np.sort(-4.0 / h**2 * np.sin(np.arange(1, n) * np.pi / (2 * n)) ** 2)
    ec = np.sort(-4.0 / h**2 * np.sin(np.arange(1, n + 1) * np.pi / (2 * n)) ** 2)
    assert np.allclose(lf, ef, rtol=1e-12, atol=0)
    assert np.allclose(lc, ec, rtol=1e-12, atol=0)


@pytest.mark.parametrize("dt", [0.05, 3.0, np.inf])
@pytest.mark.parametrize("gi", [1, 3])
def test_viscous_solve_satisfies_stencil_equation(gi, dt):
    g = GRIDS[gi]
    re = 400.0
    f = synth.random_velocity(g.nx, g.ny, g.nz, 62)
    u = stokes.viscous_solve(g, f, re, dt)
    rdt = 0.0 if np.isinf(dt) else 1.0 / dt
    lhs = rdt * u - fv.laplacian(g, u) / re
    it = ~g.wall_mask()
    assert np.all(u[g.wall_mask()] == 0.0)
    assert np.max(np.abs(lhs[it] - f[it])) <= 1e-11 * np.max(np.abs(f))


@pytest.mark.parametrize("dt", [0.2, np.inf])
def test_stokes_step_symmetric_definite_on_divergence_free(dt):
    g = GRIDS[1]
    re = 300.0
    P = simple.Projector(g)
    x, _ = P.project(synth.random_velocity(g.nx, g.ny, g.nz, 63))
    y, _ = P.project(synth.random_velocity(g.nx, g.ny, g.nz, 64))
    mu, mv, mw = g.face_volumes()
    M = g.pack(mu, mv, mw)
    sx, sy = stokes.stokes_step(g, x, re, dt), stokes.stokes_step(g, y, re, dt)
    assert simple.div_certificate(g, sx) < 1e-12
    a, b = np.sum(M * y * sx), np.sum(M * x * sy)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))
    assert np.sum(M * x * sx) > 0 and np.sum(M * y * sy) > 0


def test_stokes_step_small_dt_tends_to_dt_identity():
    g = GRIDS[0]
    re = 100.0
    x, _ = simple.Projector(g).project(synth.random_velocity(g.nx, g.ny, g.nz, 65))
    errs = []
    for dt in (1e-4, 1e-5):
        s = stokes.stokes_step(g, x, re, dt)
        errs.append(np.linalg.norm(s / dt - x) / np.linalg.norm(x))
    # first order in dt: (I/dt - A)^-1 = dt (I + dt A + ...)
    assert errs[1] < 0.2 * errs[0] and errs[0] < 0.05


def test_stokes_vector_composition():
    g = GRIDS[1]
    re = 500.0
    U = synth.random_velocity(g.nx, g.ny, g.nz, 66)
    v = synth.random_velocity(g.nx, g.ny, g.nz, 67)
    out = stokes.stokes_vector(g, U, v, re, 0.5)
    w = simple.Projector(g).krylov_vector(U, v, re)[0]
    u = stokes.viscous_solve(g, w, re, 0.5)
    assert simple.div_certificate(g, out) < 1e-12
    # out - u is a gradient (the projection removed it): its curl-free part only
    d = out - u
    assert np.linalg.norm(simple.Projector(g).project(d)[0]) <= 1e-10 * np.linalg.norm(u)
