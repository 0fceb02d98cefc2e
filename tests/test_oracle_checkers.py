"""Pins of the oracle's two judges: the divergence certificate and the Ritz residual.

Both are used to certify GPU results, so each must be shown to flag a wrong input,
not only to return small numbers on right ones.

* ``simple.div_certificate`` (reading of the "max abs divergence below 1e-12" of
  Section 3): against a brute-force loop over cells, exactly 1 for a single
  non-zero face, O(1) on an unprojected random field, at rounding level on a field
  that is divergence-free by construction (the discrete curl of an edge potential,
  built here without the projection), and raised by a single perturbed face.
* ``eigen.ritz_residual`` (the eigen-residual of eq. 7 with the oracle's operator):
  at rounding level for an exact eigenpair of the dense Krylov-vector matrix,
  exactly eps / (1 + eps) for the eigenvalue scaled by (1 + eps), exactly 2|Im lam|/|lam| for
  the conjugate eigenvalue, and large for a perturbed or foreign vector.
"""
import numpy as np
import pytest

import synth
from oracle import eigen, simple
from oracle.grid import Grid


def brute_certificate(g, vec):
    u, v, w = g.unpack(vec)
    X, Y, Z = g.X, g.Y, g.Z
    worst_net, worst_tot = 0.0, 0.0
    for k in range(g.nz):
        for j in range(g.ny):
            for i in range(g.nx):
                fl = [(u[k, j, i + 1], -u[k, j, i], Y.d[j] * Z.d[k]),
                      (v[k, j + 1, i], -v[k, j, i], X.d[i] * Z.d[k]),
                      (w[k + 1, j, i], -w[k, j, i], X.d[i] * Y.d[j])]
                net = sum((a + b) * area for a, b, area in fl)
                tot = sum((abs(a) + abs(b)) * area for a, b, area in fl)
                worst_net = max(worst_net, abs(net))
                worst_tot = max(worst_tot, tot)
    return worst_net / worst_tot


def curl_of_edge_potential(g, seed):
    """A discretely divergence-free velocity: face fluxes of the curl of a random
    potential A on cell edges (circulation of A around each face divided by the face
    area), zero on the wall-normal faces because A vanishes on wall edges."""
    X, Y, Z = g.X, g.Y, g.Z
    nx, ny, nz = g.nx, g.ny, g.nz
    rng = np.random.default_rng(seed)
    # A_x on x-edges (k face, j face, i cell), A_y on (k face, j cell, i face), A_z on (k cell, j face, i face)
    Ax = rng.uniform(-1, 1, (nz + 1, ny + 1, nx))
    Ay = rng.uniform(-1, 1, (nz + 1, ny, nx + 1))
    Az = rng.uniform(-1, 1, (nz, ny + 1, nx + 1))
    # tangential components vanish on the walls they lie in
    Ax[0], Ax[-1], Ax[:, 0], Ax[:, -1] = 0, 0, 0, 0
    Ay[0], Ay[-1], Ay[:, :, 0], Ay[:, :, -1] = 0, 0, 0, 0
    Az[:, 0], Az[:, -1], Az[:, :, 0], Az[:, :, -1] = 0, 0, 0, 0
    u = np.zeros((nz, ny, nx + 1))
    v = np.zeros((nz, ny + 1, nx))
    w = np.zeros((nz + 1, ny, nx))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx + 1):
                circ = (Az[k, j + 1, i] - Az[k, j, i]) * Z.d[k] - (Ay[k + 1, j, i] - Ay[k, j, i]) * Y.d[j]
                u[k, j, i] = circ / (Y.d[j] * Z.d[k])
    for k in range(nz):
        for j in range(ny + 1):
            for i in range(nx):
                circ = (Ax[k + 1, j, i] - Ax[k, j, i]) * X.d[i] - (Az[k, j, i + 1] - Az[k, j, i]) * Z.d[k]
                v[k, j, i] = circ / (X.d[i] * Z.d[k])
    for k in range(nz + 1):
        for j in range(ny):
            for i in range(nx):
                circ = (Ay[k, j, i + 1] - Ay[k, j, i]) * Y.d[j] - (Ax[k, j + 1, i] - Ax[k, j, i]) * X.d[i]
                w[k, j, i] = circ / (X.d[i] * Y.d[j])
    return g.pack(u, v, w)


@pytest.mark.parametrize("kind", ["uniform", "tanh", "sine"])
def test_certificate_equals_brute_force(kind):
    g = Grid.make(5, 4, 3, kind=kind)
    vec = synth.random_velocity(5, 4, 3, 21)
    assert abs(simple.div_certificate(g, vec) - brute_certificate(g, vec)) <= 1e-15


def test_certificate_single_face_is_one():
    g = Grid.make(4, 5, 6, kind="tanh")
    u, v, w = g.unpack(np.zeros(g.nvel()))
    u = u.copy()
    u[2, 3, 2] = 0.7
    vec = g.pack(u, v, w)
    assert simple.div_certificate(g, vec) == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("kind", ["uniform", "tanh"])
def test_certificate_flags_random_and_accepts_curl(kind):
    g = Grid.make(6, 5, 7, kind=kind)
    raw = synth.random_velocity(6, 5, 7, 22)
    c_raw = simple.div_certificate(g, raw)
    assert 0.05 < c_raw <= 1.0, c_raw
    sol = curl_of_edge_potential(g, 23)
    assert np.all(sol[g.wall_mask()] == 0.0)
    assert simple.div_certificate(g, sol) < 1e-14
    # the projection of the random field passes, one perturbed interior face fails
    p, _ = simple.Projector(g).project(raw)
    assert simple.div_certificate(g, p) < 1e-13
    bad = sol.copy()
    interior = np.nonzero(~g.wall_mask())[0]
    bad[interior[interior.size // 3]] += 1e-6 * np.max(np.abs(sol))
    assert simple.div_certificate(g, bad) > 1e-8


@pytest.fixture(scope="module")
def small_pair():
    """Exact eigenpairs of the dense Krylov-vector matrix on a 4^3 tanh grid with a
    random divergence-free base flow (leading complex pair and a real one if any)."""
    g = Grid.make(4, 4, 4, kind="tanh")
    proj = simple.Projector(g)
    U, _ = proj.project(synth.random_velocity(4, 4, 4, 31))
    U = 3.0 * U / np.max(np.abs(U))
    re = 200.0
    lam_s, A = eigen.dense_projected(g, U, re)
    lam, X = np.linalg.eig(A)
    it = np.nonzero(~g.wall_mask())[0]
    keep = np.argsort(np.abs(lam))[g.nx * g.ny * g.nz - 1:]
    cplx = [q for q in keep if abs(lam[q].imag) > 1e-6 * abs(lam[q])]
    assert cplx, "need a complex eigenvalue for the conjugate check"
    q = max(cplx, key=lambda q: lam[q].real)
    x = np.zeros(g.nvel(), complex)
    x[it] = X[:, q]
    return g, U, re, lam[q], x


def test_ritz_residual_exact_pair(small_pair):
    g, U, re, lam, x = small_pair
    assert eigen.ritz_residual(g, U, re, lam, x) < 1e-11


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_ritz_residual_scaled_eigenvalue(small_pair, eps):
    g, U, re, lam, x = small_pair
    r = eigen.ritz_residual(g, U, re, lam * (1 + eps), x)
    # |A x - lam (1 + eps) x| = eps |lam| |x| for an exact pair, divided by |lam (1 + eps)| |x|
    assert r == pytest.approx(eps / (1 + eps), rel=1e-6)


def test_ritz_residual_conjugate_and_perturbed_vector(small_pair):
    g, U, re, lam, x = small_pair
    r = eigen.ritz_residual(g, U, re, np.conj(lam), x)
    assert r == pytest.approx(2 * abs(lam.imag) / abs(lam), rel=1e-8)
    rng = np.random.default_rng(5)
    it = np.nonzero(~g.wall_mask())[0]
    z = np.zeros(g.nvel(), complex)
    z[it] = rng.standard_normal(it.size)
    z, _ = simple.Projector(g).project(z.real)
    xp = x + 1e-3 * np.linalg.norm(x) * z / np.linalg.norm(z)
    assert eigen.ritz_residual(g, U, re, lam, xp) > 1e-5
    assert eigen.ritz_residual(g, U, re, lam, z.astype(complex)) > 1e-2
