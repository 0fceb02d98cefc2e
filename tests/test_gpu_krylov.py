"""GPU parity of the Krylov drivers: Newton steady states and Arnoldi leading
eigenvalues against the FP64 oracle and the stored oracle spectra.

Tolerances: Newton is converged to |P R(U)|_inf <= 1e-11 on both sides, so the
base flows agree to ~1e-11 / (smallest eigenvalue ~0.7) -> 1e-9.  Arnoldi with
exact (FP64) projections must reproduce the oracle's dense eigenvalues to 1e-10
relative on the same base flow; on the GPU's own base flow the leading values
move by ~|dU| ~ 1e-10, so 1e-8 there.
"""
import os

import numpy as np
import pytest

import synth
from oracle import eigen, simple
from oracle.grid import Grid
from oracle.newton import Newton

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    a = np.loadtxt(os.path.join(GOLDEN, name))
    return a[:, 0] + 1j * a[:, 1]


def rel_match(got, ref):
    """Largest relative distance from each computed eigenvalue to the nearest
    reference value (conjugate pairs may come in either order)."""
    ref = np.asarray(ref)
    return max(float(np.min(np.abs(ref - z)) / np.abs(ref[np.argmin(np.abs(ref - z))])) for z in got)


def torch():
    import torch as t
    return t


def dev(a):
    return torch().from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch().cuda.synchronize()
    return t.cpu().numpy()


def ctx(nx, ny, nz, kind, re, alpha):
    import paper_1704_08521_amd as lk
    print(f"[case] {nx}x{ny}x{nz} {kind} re={re} alpha={alpha}", flush=True)
    c = lk.Context(nx, ny, nz)
    c.set_stretching(kind, 10.0)
    c.set_re(re)
    c.set_lid(alpha)
    return c


@pytest.mark.parametrize("case", [(8, 8, 8, "uniform", 100.0, 0.0), (10, 9, 8, "tanh", 300.0, np.pi / 4)])
def test_newton_matches_oracle(case):
    nx, ny, nz, kind, re, al = case
    c = ctx(nx, ny, nz, kind, re, al)
    hist = c.newton(tol=1e-11, max_steps=10, lin_tol=1e-10, gmres_m=100)
    print("gpu |F|:", hist)
    assert hist[-1] <= 1e-11 and len(hist) <= 9
    for a, b in zip(hist[2:-1], hist[3:]):          # quadratic once in the basin
        assert b <= 10.0 * a * a + 1e-12
    g = Grid.make(nx, ny, nz, kind=kind)
    U, ohist = Newton(g, re, al).solve(tol=1e-12)
    Ug = host(c.get_base_flow())
    assert np.max(np.abs(Ug - U)) < 1e-9 * np.max(np.abs(U))


def test_bicgstab2_handoff():
    # the BiCGstab(2) path (gmres_m = 0: BiCGstab(2) alone, the solver the paper
    # used at 100^3) on the Stokes-like first Newton step
    c = ctx(8, 8, 8, "uniform", 50.0, 0.0)
    st = c.newton_step(lin_tol=1e-10, gmres_m=0, max_vectors=3000)
    print(st)
    assert st["bicgstab"] and st["converged"]
    g = Grid.make(8)
    # one exact Newton step from U = 0 (the Stokes flow) on the oracle
    U1, _, _ = Newton(g, 50.0, 0.0).step(np.zeros(g.nvel()))
    assert np.max(np.abs(host(c.get_base_flow()) - U1)) < 1e-8 * np.max(np.abs(U1))


def test_arnoldi_8_matches_dense_spectrum():
    g = Grid.make(8)
    U, _ = Newton(g, 100.0, 0.0).solve(tol=1e-13)
    c = ctx(8, 8, 8, "uniform", 100.0, 0.0)
    c.set_base_flow(dev(U))
    out = c.arnoldi_leading(k=4, m=20, tol=1e-12, max_restarts=300, seed=7, vectors=True)
    print(out["eig"], out["resid"], out["n_vectors"])
    assert out["converged"]
    ref = gold("spectrum_8_uniform_re100_a0.txt")[: len(out["eig"]) + 1]
    assert rel_match(out["eig"], ref) < 1e-10
    assert np.all(np.diff(out["eig"].real) <= 1e-12)            # real part descending
    # Ritz vectors are eigenvectors of the oracle's operator, divergence free
    vre, vim = out["vectors"]
    for q in range(len(out["eig"])):
        x = host(vre[q]) + 1j * host(vim[q])
        assert abs(np.linalg.norm(x) - 1.0) < 1e-10
        assert eigen.ritz_residual(g, U, 100.0, out["eig"][q], x) < 1e-9
        assert simple.div_certificate(g, x.real) < 1e-11


def test_arnoldi_16_first_workload():
    # 16^3 uniform, Re = 100: GPU Newton to 1e-10, then Arnoldi (20 vectors) for 4 leading
    c = ctx(16, 16, 16, "uniform", 100.0, 0.0)
    hist = c.newton(tol=1e-10, max_steps=10, lin_tol=1e-10)
    assert hist[-1] <= 1e-10
    out = c.arnoldi_leading(k=4, m=20, tol=1e-10, max_restarts=400, seed=1)
    print(out["eig"], out["n_vectors"])
    assert out["converged"]
    ref = gold("leading_16_uniform_re100_a0.txt")
    assert rel_match(out["eig"], ref) < 1e-8


def test_arnoldi_mixed_projection_leading_eigenvalue():
    # the mixed form (float32 solves in float64 refinement to 1e-8) must keep the
    # leading eigenvalues within 1e-6 relative
    g = Grid.make(8)
    U, _ = Newton(g, 100.0, 0.0).solve(tol=1e-13)
    c = ctx(8, 8, 8, "uniform", 100.0, 0.0)
    c.set_base_flow(dev(U))
    out = c.arnoldi_leading(k=4, m=20, tol=1e-9, max_restarts=300, seed=3, precision=1, proj_tol=1e-10)
    ref = gold("spectrum_8_uniform_re100_a0.txt")[: len(out["eig"]) + 1]
    err = rel_match(out["eig"], ref)
    print("mixed Arnoldi rel. err:", err)
    assert out["converged"] and err < 1e-6


def test_arnoldi_learned_form_leading_eigenvalues():
    # the learned form inside Arnoldi: every Krylov vector starts from the network's guess
    # (an untrained seeded network; a guess that does not lower the divergence falls back to
    # the plain start) and then runs mixed passes to the projection tolerance; its fixed
    # point is the plain one, so the leading eigenvalues must match the dense spectrum to 1e-6
    import paper_1704_08521_amd as lk
    g = Grid.make(8)
    U, _ = Newton(g, 100.0, 0.0).solve(tol=1e-13)
    c = ctx(8, 8, 8, "uniform", 100.0, 0.0)
    c.set_base_flow(dev(U))
    net = lk.Net(seed=5)
    c.set_net(net)
    out = c.arnoldi_leading(k=4, m=20, tol=1e-9, max_restarts=300, seed=3, precision=lk.LEARNED, proj_tol=1e-10,
                            vectors=True)
    ref = gold("spectrum_8_uniform_re100_a0.txt")[: len(out["eig"]) + 1]
    err = rel_match(out["eig"], ref)
    print("learned Arnoldi rel. err:", err, "vectors", out["n_vectors"])
    assert out["converged"] and err < 1e-6
    vre, vim = out["vectors"]
    for q in range(len(out["eig"])):
        x = host(vre[q]) + 1j * host(vim[q])
        assert eigen.ritz_residual(g, U, 100.0, out["eig"][q], x) < 1e-6
