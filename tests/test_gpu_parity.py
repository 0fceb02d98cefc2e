"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: stencils, divergence and correction are a handful of rounded
operations per output, so they must agree to 1e-12 of the field's largest
value.  The tensor-product Poisson solve applies six dense n x n transforms
(error ~ n eps cond(S), cond(S) = sqrt(max d / min d) <= 4 here), so 1e-11.
The Krylov vector must match the oracle to 1e-10 relative (the FP64 target);
the mixed form to 1e-6, with its SIMPLE certificate rho <= tol.
"""
import math

import numpy as np
import pytest

import synth
from oracle import fv, poisson, simple
from oracle.grid import Grid

pytestmark = pytest.mark.gpu

CASES = [(8, 8, 8, "uniform"), (17, 19, 23, "tanh"), (33, 20, 27, "sine"), (2, 3, 2, "uniform"),
         (64, 64, 64, "tanh")]


def torch():
    import torch as t
    return t


def ctx_for(nx, ny, nz, kind, re=700.0, alpha=0.3, seed=1):
    import paper_1704_08521_amd as lk
    print(f"[case] {nx}x{ny}x{nz} {kind} re={re} alpha={alpha} seed={seed}", flush=True)
    c = lk.Context(nx, ny, nz)
    c.set_stretching(kind, 10.0)
    c.set_re(re)
    c.set_lid(alpha)
    g = Grid.make(nx, ny, nz, kind=kind)
    U = synth.random_velocity(nx, ny, nz, seed)
    c.set_base_flow(dev(U))
    return c, g, U


def dev(a):
    return torch().from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch().cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("case", CASES)
def test_grid_faces_match(case):
    nx, ny, nz, kind = case
    c, g, _ = ctx_for(nx, ny, nz, kind)
    xf, yf, zf = c.get_grid()
    assert np.allclose(xf, g.X.xf, atol=1e-15) and np.allclose(zf, g.Z.xf, atol=1e-15)


@pytest.mark.parametrize("case", CASES)
def test_jacobian_stencil(case):
    nx, ny, nz, kind = case
    c, g, U = ctx_for(nx, ny, nz, kind)
    v = synth.random_velocity(nx, ny, nz, 2)
    w = host(c.jacobian_apply(dev(v)))
    ref = fv.jacobian_apply(g, U, v, 700.0)
    assert rel(w, ref) < 1e-12
    assert np.all(w[g.wall_mask()] == 0.0)


@pytest.mark.parametrize("case", CASES)
def test_residual_stencil(case):
    nx, ny, nz, kind = case
    c, g, U = ctx_for(nx, ny, nz, kind)
    R = host(c.residual(dev(U)))
    assert rel(R, fv.residual(g, U, 700.0, 0.3)) < 1e-12


def test_inputs_wall_faces_are_ignored():
    c, g, U = ctx_for(9, 7, 8, "tanh")
    v = synth.random_velocity(9, 7, 8, 2)
    dirty = v + g.wall_mask() * 5.0
    assert np.array_equal(host(c.jacobian_apply(dev(dirty))), host(c.jacobian_apply(dev(v))))


@pytest.mark.parametrize("case", CASES)
def test_divergence_and_correction(case):
    nx, ny, nz, kind = case
    c, g, _ = ctx_for(nx, ny, nz, kind)
    v = synth.random_velocity(nx, ny, nz, 3)
    r_t, nrm = c.divergence(dev(v))
    r = host(r_t).reshape(nz, ny, nx)
    ref = fv.divergence(g, v)
    assert rel(r, ref) < 1e-12
    assert math.isclose(nrm, simple.vnorm(g, ref), rel_tol=1e-12)
    phi = synth.random_cells(nx, ny, nz, 4)
    vv, pp = c.correct(dev(v), dev(phi.ravel()))
    assert rel(host(vv), fv.zero_walls(g, v) - fv.gradient(g, phi)) < 1e-12
    assert np.array_equal(host(pp), phi.ravel())


@pytest.mark.parametrize("case", CASES)
def test_simple_pass_certificate_and_second_pass(case):
    # one SIMPLE pass: its certificate equals the separate divergence norm of the stored
    # v, and v, p are the plain correction; a second (FP32) pass solves with D v of the first
    nx, ny, nz, kind = case
    c, g, _ = ctx_for(nx, ny, nz, kind)
    w_h = synth.random_velocity(nx, ny, nz, 9)
    w = dev(w_h)
    _, n0 = c.divergence(w)
    for prec, rtol in ((1, 1e-9), (0, 1e-6)):
        vo, po, st = c.project(w, precision=prec, tol=0.0, max_iter=1)
        _, n1 = c.divergence(vo)
        print(f"precision {prec}: rho {st['rho']:.6e} separate {n1 / n0:.6e}")
        assert st["iterations"] == 1 and math.isclose(st["rho"], n1 / n0, rel_tol=rtol)
        phi = host(po).reshape(nz, ny, nx)
        assert rel(host(vo), fv.zero_walls(g, w_h) - fv.gradient(g, phi)) < 1e-12
    vo, _, st = c.project(w, precision=1, tol=0.0, max_iter=2)
    vo1, po1, _ = c.project(w, precision=1, tol=0.0, max_iter=1)
    r1, _ = c.divergence(vo1)
    phi2 = c.poisson_solve(r1, precision=1)
    ref2 = host(vo1) - fv.zero_walls(g, fv.gradient(g, host(phi2).reshape(nz, ny, nx)))
    assert st["iterations"] == 2 and rel(host(vo), ref2) < 1e-12


@pytest.mark.parametrize("case", CASES)
def test_poisson_solve(case):
    nx, ny, nz, kind = case
    c, g, _ = ctx_for(nx, ny, nz, kind)
    r = synth.random_cells(nx, ny, nz, 5)
    V = g.volumes()
    r = r - np.sum(V * r) / np.sum(V)
    ref = poisson.PoissonFD(g).solve(r)
    phi = host(c.poisson_solve(dev(r.ravel()))).reshape(nz, ny, nx)
    assert rel(phi, ref) < 1e-11
    phi32 = host(c.poisson_solve(dev(r.ravel()), precision=1)).reshape(nz, ny, nx)
    assert rel(phi32, ref) < 1e-4


@pytest.mark.parametrize("case", CASES)
def test_krylov_vector_fp64(case):
    nx, ny, nz, kind = case
    c, g, U = ctx_for(nx, ny, nz, kind)
    v = synth.random_velocity(nx, ny, nz, 6)
    vo, po, st = c.krylov_vector(dev(v), tol=1e-10)
    ref_v, ref_p = simple.Projector(g).krylov_vector(U, v, 700.0)
    print(f"fp64: iterations={st['iterations']} rho={st['rho']:.3e}")
    assert st["converged"] and st["iterations"] <= 2 and st["rho"] < 1e-10
    assert rel(host(vo), ref_v) < 1e-10
    assert rel(host(po).reshape(nz, ny, nx), ref_p) < 1e-10
    assert simple.div_certificate(g, host(vo)) < 1e-12


@pytest.mark.parametrize("case", CASES)
def test_krylov_vector_mixed(case):
    nx, ny, nz, kind = case
    c, g, U = ctx_for(nx, ny, nz, kind)
    v = synth.random_velocity(nx, ny, nz, 7)
    vo, po, st = c.krylov_vector(dev(v), precision=1, tol=1e-8)
    ref_v, _ = simple.Projector(g).krylov_vector(U, v, 700.0)
    assert st["converged"] and st["rho"] <= 1e-8
    err = rel(host(vo), ref_v)
    print(f"mixed: iterations={st['iterations']} rho={st['rho']:.3e} rel.err vs oracle={err:.3e}")
    assert err < 1e-6


def test_zero_and_nonfinite_inputs():
    import paper_1704_08521_amd as lk
    c, g, U = ctx_for(6, 5, 4, "tanh")
    zero = np.zeros(g.nvel())
    vo, po, st = c.project(dev(zero))
    assert st["converged"] and np.all(host(vo) == 0) and np.all(host(po) == 0)
    bad = synth.random_velocity(6, 5, 4, 1)
    interior = np.nonzero(~g.wall_mask())[0]
    bad[interior[interior.size // 2]] = np.nan
    with pytest.raises(lk.LidKrylovError):
        c.project(dev(bad))


def test_notconv_reported():
    c, g, U = ctx_for(12, 10, 8, "tanh")
    v = synth.random_velocity(12, 10, 8, 8)
    # one mixed pass cannot reach 1e-14
    _, _, st = c.krylov_vector(dev(v), precision=1, tol=1e-14, max_iter=1)
    assert not st["converged"] and st["iterations"] == 1


def test_full_size_krylov_vector_200():
    # the benchmark's workload: 200^3 tanh-10, Re = 1900, alpha = 0, full comparison
    nx = 200
    c, g, U = ctx_for(nx, nx, nx, "tanh", re=1900.0, alpha=0.0, seed=11)
    v = synth.random_velocity(nx, nx, nx, 12)
    vo, po, st = c.krylov_vector(dev(v), tol=1e-8)
    assert st["converged"] and st["rho"] <= 1e-8
    ref_v, ref_p = simple.Projector(g).krylov_vector(U, v, 1900.0)
    assert rel(host(vo), ref_v) < 1e-10
    vo32, _, st32 = c.krylov_vector(dev(v), precision=1, tol=1e-8)
    assert st32["converged"] and rel(host(vo32), ref_v) < 1e-6


# Grids without mirror symmetry (seeded random widths) use the full transforms; mixed
# cases combine a symmetric (uniform) axis with asymmetric ones.
def asym_faces(n, seed):
    rng = np.random.default_rng(seed)
    f = np.concatenate([[0.0], np.cumsum(0.5 + rng.random(n))])
    return f / f[-1]


ASYM = [((12, 9, 10), (True, False, True)), ((7, 8, 9), (False, False, False)),
        ((16, 16, 15), (False, True, True))]


def ctx_faces(dims, sym, re=650.0, alpha=0.2, seed=3):
    import paper_1704_08521_amd as lk
    print(f"[case] {dims} symmetric axes {sym}", flush=True)
    faces = [np.linspace(0.0, 1.0, n + 1) if s else asym_faces(n, 40 + a) for a, (n, s) in enumerate(zip(dims, sym))]
    c = lk.Context(*dims)
    c.set_grid(*faces)
    c.set_re(re)
    c.set_lid(alpha)
    g = Grid(*faces)
    U = synth.random_velocity(*dims, seed)
    c.set_base_flow(dev(U))
    return c, g, U


@pytest.mark.parametrize("case", ASYM)
def test_poisson_solve_asymmetric_grids(case):
    dims, sym = case
    c, g, _ = ctx_faces(dims, sym)
    nx, ny, nz = dims
    r = synth.random_cells(nx, ny, nz, 7)
    V = g.volumes()
    r = r - np.sum(V * r) / np.sum(V)
    ref = poisson.PoissonFD(g).solve(r)
    phi = host(c.poisson_solve(dev(r.ravel()))).reshape(nz, ny, nx)
    assert rel(phi, ref) < 1e-11
    phi32 = host(c.poisson_solve(dev(r.ravel()), precision=1)).reshape(nz, ny, nx)
    assert rel(phi32, ref) < 1e-4


@pytest.mark.parametrize("case", ASYM)
def test_krylov_vector_asymmetric_grids(case):
    dims, sym = case
    c, g, U = ctx_faces(dims, sym)
    v = synth.random_velocity(*dims, 8)
    vo, po, st = c.krylov_vector(dev(v), tol=1e-10)
    ref_v, _ = simple.Projector(g).krylov_vector(U, v, 650.0)
    assert st["converged"] and rel(host(vo), ref_v) < 1e-10


# Both routes of the pressure solve, each selected explicitly (TPT, the default: transforms
# along y and z, tridiagonal solves along x; TPF: transforms along x, y and z) against the
# same oracle solves, on the symmetric, odd and asymmetric grids and at 200^3.
@pytest.mark.parametrize("method", ["tpt", "tpf"])
@pytest.mark.parametrize("case", CASES)
def test_poisson_solve_each_route(case, method):
    nx, ny, nz, kind = case
    c, g, U = ctx_for(nx, ny, nz, kind)
    c.set_poisson_method(method)
    r = synth.random_cells(nx, ny, nz, 5)
    V = g.volumes()
    r = r - np.sum(V * r) / np.sum(V)
    ref = poisson.PoissonFD(g).solve(r)
    phi = host(c.poisson_solve(dev(r.ravel()))).reshape(nz, ny, nx)
    assert rel(phi, ref) < 1e-11
    phi32 = host(c.poisson_solve(dev(r.ravel()), precision=1)).reshape(nz, ny, nx)
    assert rel(phi32, ref) < 1e-4
    v = synth.random_velocity(nx, ny, nz, 6)
    vo, po, st = c.krylov_vector(dev(v), tol=1e-10)
    ref_v, ref_p = simple.Projector(g).krylov_vector(U, v, 700.0)
    assert st["converged"] and st["iterations"] <= 2
    assert rel(host(vo), ref_v) < 1e-10 and rel(host(po).reshape(nz, ny, nx), ref_p) < 1e-10


@pytest.mark.parametrize("method", ["tpt", "tpf"])
@pytest.mark.parametrize("case", ASYM)
def test_poisson_solve_each_route_asymmetric_grids(case, method):
    dims, sym = case
    c, g, _ = ctx_faces(dims, sym)
    c.set_poisson_method(method)
    nx, ny, nz = dims
    r = synth.random_cells(nx, ny, nz, 7)
    V = g.volumes()
    r = r - np.sum(V * r) / np.sum(V)
    ref = poisson.PoissonFD(g).solve(r)
    phi = host(c.poisson_solve(dev(r.ravel()))).reshape(nz, ny, nx)
    assert rel(phi, ref) < 1e-11
    phi32 = host(c.poisson_solve(dev(r.ravel()), precision=1)).reshape(nz, ny, nx)
    assert rel(phi32, ref) < 1e-4


@pytest.mark.parametrize("n", [1000, 513, 300, 128, 100, 65])
def test_tpt_line_lengths(n):
    # every rows-per-lane instance of the tridiagonal pass (2 rows: 65-128 cells, 8: 257-512,
    # 16: 513-1024; 1 and 4 are covered by the grids above) and the x transforms of the TPF
    # route on a thin grid, each against the oracle's exact solve
    c, g, _ = ctx_for(n, 3, 4, "tanh")
    r = synth.random_cells(n, 3, 4, 17)
    V = g.volumes()
    r = r - np.sum(V * r) / np.sum(V)
    ref = poisson.PoissonFD(g).solve(r).ravel()
    rd = dev(r.ravel())
    c.set_poisson_method("tpf")
    phi_f = host(c.poisson_solve(rd))
    c.set_poisson_method("tpt")
    phi_t = host(c.poisson_solve(rd))
    print(f"n={n}: tpt {rel(phi_t, ref):.2e} tpf {rel(phi_f, ref):.2e}")
    # both sides round n-term inner products along the long line: 1e-13 n beyond n = 100
    # (the derivation is in test_gpu_instances)
    bound = max(1e-11, 1e-13 * n)
    assert rel(phi_t, ref) < bound and rel(phi_f, ref) < bound


def test_routes_agree_full_size_200():
    # the benchmark's workload: TPT and TPF on the same right side against the oracle's
    # solve, and the TPT Krylov vector against the oracle, full fields
    nx = 200
    c, g, U = ctx_for(nx, nx, nx, "tanh", re=1900.0, alpha=0.0, seed=11)
    r = synth.random_cells(nx, nx, nx, 13)
    V = g.volumes()
    r = r - np.sum(V * r) / np.sum(V)
    rd = dev(r.ravel())
    ref = poisson.PoissonFD(g).solve(r).ravel()
    c.set_poisson_method("tpf")
    phi_f = host(c.poisson_solve(rd))
    c.set_poisson_method("tpt")
    phi_t = host(c.poisson_solve(rd))
    print(f"at 200^3: TPT vs oracle {rel(phi_t, ref):.3e}, TPF vs oracle {rel(phi_f, ref):.3e}")
    assert rel(phi_t, ref) < 1e-11 and rel(phi_f, ref) < 1e-11
    v = synth.random_velocity(nx, nx, nx, 12)
    vo, _, st = c.krylov_vector(dev(v), tol=1e-8)
    assert st["converged"] and st["rho"] <= 1e-8
    ref_v, _ = simple.Projector(g).krylov_vector(U, v, 1900.0)
    assert rel(host(vo), ref_v) < 1e-10


def test_poisson_method_rejects_unknown():
    from paper_1704_08521_amd import LidKrylovError
    c, g, _ = ctx_for(8, 8, 8, "uniform")
    with pytest.raises(LidKrylovError):
        c._check(c.lib.lc_set_poisson_method(c._h, 7))
