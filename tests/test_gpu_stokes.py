"""GPU parity of the Stokes-preconditioned (time-stepper) Krylov vectors against the oracle.

The viscous step is six dense 1D transforms per component, like the pressure solve, so it
must match the oracle's sparse direct solve to 1e-11 relative (the bound of
test_gpu_parity's Poisson cases); the Stokes step and the Stokes-preconditioned Krylov
vector add one exact projection each, 1e-10 (the FP64 Krylov-vector bound).  Newton with
the Stokes step as right preconditioner must reach the oracle's steady state like the
unpreconditioned solver (1e-9, see test_gpu_krylov).
"""
import numpy as np
import pytest

import synth
from oracle import stokes
from oracle.grid import Grid
from oracle.newton import Newton

pytestmark = pytest.mark.gpu


def torch():
    import torch as t
    return t


def dev(a):
    return torch().from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch().cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def asym_faces(n, seed):
    rng = np.random.default_rng(seed)
    f = np.concatenate([[0.0], np.cumsum(0.5 + rng.random(n))])
    return f / f[-1]


# (dims, kind): symmetric grids take the folded transforms (matrix cores for half lengths
# <= 128, of both the n-cell and the (n+1)-face factors), "asym" grids the full ones, and the
# thin grids the larger row-tile instances and the vector-FMA path (n + 1 > 256 faces)
CASES = [((8, 8, 8), "uniform"), ((9, 7, 6), "tanh"), ((12, 10, 11), "sine"), ((7, 6, 9), "asym"),
         ((4, 100, 3), "tanh"), ((3, 4, 150), "tanh"), ((256, 3, 4), "tanh"), ((3, 300, 4), "tanh")]


def make(dims, kind, re=400.0, alpha=0.2):
    import paper_1704_08521_amd as lk
    print(f"[case] {dims} {kind}", flush=True)
    c = lk.Context(*dims)
    if kind == "asym":
        fs = [asym_faces(n, 70 + a) for a, n in enumerate(dims)]
        c.set_grid(*fs)
        g = Grid(*fs)
    else:
        c.set_stretching(kind, 10.0)
        g = Grid.make(*dims, kind=kind, ratio=10.0)
    c.set_re(re)
    c.set_lid(alpha)
    return c, g


@pytest.mark.parametrize("dt", [0.3, float("inf")])
@pytest.mark.parametrize("case", CASES)
def test_viscous_solve(case, dt):
    dims, kind = case
    c, g = make(dims, kind)
    f = synth.random_velocity(*dims, 81)
    u = host(c.viscous_solve(dev(f), dt))
    ref = stokes.viscous_solve(g, f, 400.0, dt)
    e = rel(u, ref)
    print(f"  viscous dt={dt}: {e:.2e}")
    assert e < 1e-11
    assert np.all(u[g.wall_mask()] == 0.0)


@pytest.mark.parametrize("case", CASES[:4])
def test_stokes_step_and_vector(case):
    dims, kind = case
    c, g = make(dims, kind)
    U = synth.random_velocity(*dims, 82)
    c.set_base_flow(dev(U))
    f = synth.random_velocity(*dims, 83)
    for dt in (0.3, float("inf")):
        u, st = c.stokes_step(dev(f), dt, tol=1e-12)
        assert st["converged"]
        e1 = rel(host(u), stokes.stokes_step(g, f, 400.0, dt))
        o, st2 = c.stokes_vector(dev(f), dt, tol=1e-12)
        assert st2["converged"]
        e2 = rel(host(o), stokes.stokes_vector(g, U, f, 400.0, dt))
        print(f"  dt={dt}: step {e1:.2e} vector {e2:.2e}")
        assert e1 < 1e-10 and e2 < 1e-10


def test_stokes_bad_arguments():
    import paper_1704_08521_amd as lk
    c, g = make((6, 5, 4), "tanh")
    f = dev(synth.random_velocity(6, 5, 4, 84))
    for dt in (0.0, -1.0, float("nan")):
        with pytest.raises(lk.LidKrylovError):
            c.viscous_solve(f, dt)
    with pytest.raises(lk.LidKrylovError):
        c.viscous_solve(f, 1.0, out=f)
    with pytest.raises(lk.LidKrylovError):
        c.set_stokes_precond(-1.0)


@pytest.mark.parametrize("dt", [float("inf"), 0.5])
@pytest.mark.parametrize("case", [(8, 8, 8, "uniform", 100.0, 0.0), (10, 9, 8, "tanh", 300.0, np.pi / 4)])
def test_preconditioned_newton_matches_oracle(case, dt):
    import paper_1704_08521_amd as lk
    nx, ny, nz, kind, re, al = case
    print(f"[case] Newton {case} dt={dt}", flush=True)
    c = lk.Context(nx, ny, nz)
    c.set_stretching(kind, 10.0)
    c.set_re(re)
    c.set_lid(al)
    c.set_stokes_precond(dt)
    hist, vecs = [], []
    for _ in range(10):
        _, r = c.newton_residual()
        hist.append(r)
        if r <= 1e-11:
            break
        st = c.newton_step(lin_tol=1e-10, gmres_m=100, max_vectors=5000)
        vecs.append(st["n_vectors"])
    print("gpu |F|:", hist, "vectors per step:", vecs)
    assert hist[-1] <= 1e-11 and len(hist) <= 9
    g = Grid.make(nx, ny, nz, kind=kind)
    U, _ = Newton(g, re, al).solve(tol=1e-12)
    Ug = host(c.get_base_flow())
    assert np.max(np.abs(Ug - U)) < 1e-9 * np.max(np.abs(U))
