"""Every compiled instance of the pressure-solve kernels against the FP64 oracle.

The tensor-product solve (Section 3, TPT and TPF) dispatches on the line length of
each axis:

* mirror-symmetric axes, half length he = ceil(n/2) <= 128: matrix-core transforms
  with RT = ceil(he/16) row tiles (RT 1..8: n up to 32, 64, 96, 128, 160, 192, 224, 256),
  the RT = 8 instance at two waves per SIMD;
* mirror-symmetric axes with n > 256: folded vector-FMA transforms (row tiles 10, 13, 16
  and the several-block case of he > 256);
* axes without mirror symmetry: full vector-FMA transforms (tiles 1, 2, 4, 8, 10, 7, 16
  by line length);
* the TPT tridiagonal pass along x with 1, 2, 4, 8 or 16 rows per lane (n up to 64,
  128, 256, 512, 1024).

Each case puts the long axis on x (right transforms and the tridiagonal pass), on y
(segmented left transforms) or on z (left transforms with the eigenvalue division),
keeps the other two axes short, and compares both routes with the oracle's exact solve.

Tolerances (max |error| / max |oracle|).  Both sides round every n-term inner product of
their dense line transforms (and the oracle its own eigen-decomposition), so the FP64
difference grows with the longest line n: 1e-11 up to n = 100, then 1e-13 n (measured:
2e-11 at n = 420..513, 5e-11 at n = 1000 -- about 400 n u64, half the bound).  FP32: 1e-4,
except that the tridiagonal x pass of the TPT route accumulates its FP32 elimination and
back-substitution along the whole line (and the zero-mode line is recentred after it), so
there 2e-6 n_x (measured 1.1e-4 at 150, 1.5e-3 at 1000, i.e. about 25 n u32); in the mixed
form this only changes how fast the FP64 refinement converges, not its fixed point.
A few thin grids also run the whole Krylov vector (1e-10).
"""
import numpy as np
import pytest

import synth
from oracle import poisson, simple
from oracle.grid import Grid

pytestmark = pytest.mark.gpu

SYM_LENGTHS = [80, 100, 150, 170, 210, 256, 300, 420, 513, 1000]
ASYM_LENGTHS = [12, 20, 40, 100, 150, 170, 300]


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


def make(dims, long_axis, symmetric, re=800.0, alpha=0.25):
    import paper_1704_08521_amd as lk
    from oracle.grid import faces as oracle_faces
    fs = []
    for a, n in enumerate(dims):
        if a == long_axis and not symmetric:
            fs.append(asym_faces(n, 100 + n))
        else:
            fs.append(oracle_faces(n, "tanh", 10.0))
    print(f"[case] dims {dims} long axis {long_axis} {'tanh' if symmetric else 'asymmetric'}", flush=True)
    c = lk.Context(*dims)
    c.set_grid(*fs)
    c.set_re(re)
    c.set_lid(alpha)
    return c, Grid(*fs)


def dims_for(n, axis):
    d = [3, 4, 5]
    d[axis] = n
    return tuple(d)


def bound64(g):
    return max(1e-11, 1e-13 * max(g.nx, g.ny, g.nz))


def bound32(g, method):
    return max(1e-4, 2e-6 * g.nx) if method == "tpt" else 1e-4


def check_routes(c, g, seed):
    nx, ny, nz = g.nx, g.ny, g.nz
    r = synth.random_cells(nx, ny, nz, seed)
    V = g.volumes()
    r = r - np.sum(V * r) / np.sum(V)
    ref = poisson.PoissonFD(g).solve(r)
    rd = dev(r.ravel())
    for method in ("tpt", "tpf"):
        c.set_poisson_method(method)
        phi = host(c.poisson_solve(rd)).reshape(nz, ny, nx)
        phi32 = host(c.poisson_solve(rd, precision=1)).reshape(nz, ny, nx)
        e64, e32 = rel(phi, ref), rel(phi32, ref)
        print(f"  {method}: fp64 {e64:.2e} fp32 {e32:.2e}", flush=True)
        assert e64 < bound64(g), (method, e64)
        assert e32 < bound32(g, method), (method, e32)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n", SYM_LENGTHS)
def test_symmetric_axis_instances(n, axis):
    c, g = make(dims_for(n, axis), axis, True)
    check_routes(c, g, 300 + n + axis)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n", ASYM_LENGTHS)
def test_asymmetric_axis_instances(n, axis):
    c, g = make(dims_for(n, axis), axis, False)
    check_routes(c, g, 500 + n + axis)


# Thin grids whose two long axes take the instances of the benchmark-family grids:
# RT 4 (100^3), RT 5 (130 and 150^3), RT 8 at two waves per SIMD (256^3), and a folded
# vector-FMA axis (n > 256) -- the whole Krylov vector on both routes.
THIN = [(4, 100, 100), (4, 150, 150), (3, 130, 130), (3, 256, 256), (300, 3, 40), (40, 300, 3)]


@pytest.mark.parametrize("dims", THIN)
def test_thin_grid_krylov_vector(dims):
    import paper_1704_08521_amd as lk
    nx, ny, nz = dims
    print(f"[case] thin {dims}", flush=True)
    c = lk.Context(nx, ny, nz)
    c.set_stretching("tanh", 10.0)
    c.set_re(1500.0)
    c.set_lid(0.0)
    g = Grid.make(nx, ny, nz, kind="tanh", ratio=10.0)
    U = synth.random_velocity(nx, ny, nz, 41)
    c.set_base_flow(dev(U))
    v = synth.random_velocity(nx, ny, nz, 42)
    ref_v, ref_p = simple.Projector(g).krylov_vector(U, v, 1500.0)
    for method in ("tpt", "tpf"):
        c.set_poisson_method(method)
        vo, po, st = c.krylov_vector(dev(v), tol=1e-10)
        ev, ep = rel(host(vo), ref_v), rel(host(po).reshape(nz, ny, nx), ref_p)
        print(f"  {method}: v {ev:.2e} p {ep:.2e} rho {st['rho']:.2e}", flush=True)
        assert st["converged"] and ev < 1e-10 and ep < 1e-10
        vm, _, stm = c.krylov_vector(dev(v), precision=1, tol=1e-8)
        assert stm["converged"] and rel(host(vm), ref_v) < 1e-6
