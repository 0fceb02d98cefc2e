"""Pins of the oracle's Poisson solve, projection, Newton and eigenvalue paths."""
import os

import numpy as np
import pytest

import synth
from oracle import eigen, fv, poisson, simple
from oracle.grid import Grid
from oracle.newton import Newton
from tests import mms

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_spectrum(name):
    a = np.loadtxt(os.path.join(GOLDEN, name))
    return a[:, 0] + 1j * a[:, 1]


# ------------------------------------------------------------------- Poisson
@pytest.mark.parametrize("kind", ["uniform", "sine", "tanh"])
def test_poisson_manufactured_second_order(kind):
    errs = []
    for n in (16, 32, 64):
        g = Grid.make(n, kind=kind)
        x, y, z = mms.cell_points(g)
        ex = mms.cos3(x, y, z)
        phi = poisson.PoissonFD(g).solve(-3 * np.pi ** 2 * ex)
        V = g.volumes()
        errs.append(np.max(np.abs(phi - (ex - np.sum(V * ex) / np.sum(V)))))
    o = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(o > 1.9), errs


def test_poisson_equals_dense_least_squares():
    # brute force: the assembled D G matrix, minimum-norm least squares, then the
    # volume-weighted mean removed
    g = Grid.make(4, 5, 6, kind="tanh")
    n = 4 * 5 * 6
    A = np.empty((n, n))
    for c in range(n):
        e = np.zeros(n); e[c] = 1.0
        A[:, c] = poisson.apply_DG(g, e.reshape(6, 5, 4)).ravel()
    r = synth.random_cells(4, 5, 6, 5)
    V = g.volumes()
    r = r - np.sum(V * r) / np.sum(V)          # compatible right side
    ls = np.linalg.lstsq(A, r.ravel(), rcond=None)[0].reshape(6, 5, 4)
    ls -= np.sum(V * ls) / np.sum(V)
    fd = poisson.PoissonFD(g).solve(r)
    assert np.max(np.abs(fd - ls)) < 1e-12 * max(1.0, np.max(np.abs(ls)))
    assert abs(np.sum(V * fd)) < 1e-14


# ---------------------------------------------------------------- projection
def test_projection_properties():
    g = Grid.make(9, 7, 8, kind="tanh")
    P = simple.Projector(g)
    w = synth.random_velocity(9, 7, 8, 7)
    pw, phi = P.project(w)
    assert simple.div_certificate(g, pw) < 1e-12          # Section 3: div < 1e-12 (TPF)
    assert np.max(np.abs(P.project(pw)[0] - pw)) < 1e-12 * np.max(np.abs(pw))   # idempotent
    q = synth.random_cells(9, 7, 8, 8)
    assert np.max(np.abs(P.project(fv.gradient(g, q))[0])) < 1e-10   # P G = 0
    assert np.all(pw[g.wall_mask()] == 0.0)
    # P is orthogonal in the M_u inner product: <P w, w - P w>_M = 0
    mu, mv, mw = g.face_volumes()
    M = g.pack(mu, mv, mw)
    assert abs(np.sum(M * pw * (w - pw))) < 1e-12 * np.sum(M * w * w)


@pytest.mark.parametrize("kind", ["uniform", "tanh"])
def test_projection_manufactured(kind):
    u_ex = mms.psi_velocity()
    grad_q = [lambda x, y, z, a=a: mms.d(mms.cos3, a, x, y, z) for a in range(3)]
    errs = []
    for n in (12, 24, 48):
        g = Grid.make(n, kind=kind)
        w = mms.sample(g, [lambda x, y, z, c=c: u_ex[c](x, y, z) + grad_q[c](x, y, z) for c in range(3)])
        pw, _ = simple.Projector(g).project(w)
        errs.append(np.max(np.abs(pw - mms.sample(g, u_ex))))
    o = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert o[-1] > 1.8, errs


def test_simple_loop_matches_projection_in_one_pass():
    g = Grid.make(8, 6, 7, kind="sine")
    P = simple.Projector(g)
    U = synth.random_velocity(8, 6, 7, 1)
    v = synth.random_velocity(8, 6, 7, 2)
    w = fv.jacobian_apply(g, U, v, 400.0)
    vl, pl, its = P.simple_loop(w)
    vp, pp = P.krylov_vector(U, v, 400.0)
    assert its <= 2
    assert np.max(np.abs(vl - vp)) < 1e-11 * np.max(np.abs(vp))
    assert np.max(np.abs(pl - pp)) < 1e-11 * np.max(np.abs(pp))
    # eq. 8: v' = w - grad p'
    assert np.max(np.abs(vp - (fv.zero_walls(g, w) - fv.gradient(g, pp)))) < 1e-12 * np.max(np.abs(w))


# -------------------------------------------------------------------- Newton
def test_newton_quadratic_convergence():
    g = Grid.make(8)
    U, hist = Newton(g, 100.0, 0.0).solve(tol=1e-13)
    assert hist[-1] < 1e-13
    # quadratic: |F_{k+1}| <= C |F_k|^2 once in the basin
    for a, b in zip(hist[2:-1], hist[3:]):
        assert b <= 2.0 * a * a + 1e-13, hist
    assert len(hist) <= 8          # Section 3: 6-8 Newton iterations


def test_newton_manufactured_steady_state_second_order():
    re = 50.0
    u_ex = mms.psi_velocity()

    def forcing(g):
        # f = (u.grad)u - Re^-1 Lap u + grad p, p = cos(pi x) cos(pi y) cos(pi z)
        out = []
        for c in range(3):
            x, y, z = mms.face_points(g, c)
            adv = sum(u_ex[a](x, y, z) * mms.d(u_ex[c], a, x, y, z) for a in range(3))
            lap = sum(mms.d2(u_ex[c], a, x, y, z) for a in range(3))
            out.append(adv - lap / re + mms.d(mms.cos3, c, x, y, z))
        return g.pack(*out)

    errs = []
    for n in (8, 16):
        g = Grid.make(n)
        nw = Newton(g, re, None, forcing=forcing(g))
        U, hist = nw.solve(tol=1e-11)
        assert hist[-1] < 1e-11
        errs.append(np.max(np.abs(U - mms.sample(g, u_ex))))
    assert errs[0] / errs[1] > 3.0, errs


def test_base_flow_symmetries():
    g = Grid.make(8, kind="tanh")
    U, _ = Newton(g, 100.0, 0.0).solve(tol=1e-12)
    u, v, w = g.unpack(U)
    # alpha = 0: reflection y -> 1 - y with v odd
    assert np.max(np.abs(u - u[:, ::-1, :])) < 1e-12
    assert np.max(np.abs(v + v[:, ::-1, :])) < 1e-12
    assert np.max(np.abs(w - w[:, ::-1, :])) < 1e-12
    U, _ = Newton(g, 100.0, np.pi / 4).solve(tol=1e-12)
    u, v, w = g.unpack(U)
    # alpha = 45 deg: reflection x <-> y exchanging u and v
    assert np.max(np.abs(u - np.transpose(v, (0, 2, 1)))) < 1e-12
    assert np.max(np.abs(w - np.transpose(w, (0, 2, 1)))) < 1e-12


# ---------------------------------------------------------------- eigenvalues
@pytest.fixture(scope="module")
def base8():
    g = Grid.make(8)
    U, _ = Newton(g, 100.0, 0.0).solve(tol=1e-13)
    return g, U


def test_dense_constructions_match_golden_spectrum(base8):
    g, U = base8
    gold = load_spectrum("spectrum_8_uniform_re100_a0.txt")
    ld, _ = eigen.dense_projected(g, U, 100.0)
    ln = eigen.nullspace(g, U, 100.0)
    assert ld.size == ln.size == gold.size == 833
    assert eigen.match_distance(gold, ld) < 1e-10 * np.max(np.abs(gold))
    assert eigen.match_distance(gold, ln) < 1e-10 * np.max(np.abs(gold))


def test_arpack_leading_matches_dense(base8):
    g, U = base8
    gold = load_spectrum("spectrum_8_uniform_re100_a0.txt")
    lam = eigen.arpack(g, U, 100.0, k=4, ncv=20, tol=1e-12)
    assert np.max(np.abs(lam[:3] - gold[:3])) < 1e-10


def test_stokes_limit_spectrum_real_negative():
    # U = 0: P Lap/Re is self-adjoint and negative definite on S in the M_u product
    g = Grid.make(6, 7, 5, kind="tanh")
    lam, _ = eigen.dense_projected(g, np.zeros(g.nvel()), 10.0)
    assert np.max(np.abs(lam.imag)) < 1e-10
    assert np.max(lam.real) < 0.0
