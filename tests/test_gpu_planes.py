"""GPU parity of the plane projections and their potentials (Section 4, eqs. 11-17).

Small grids: element-wise against the dense per-plane oracle (oracle.planes), out and
psi to 1e-11 of their largest value, on the default route (the planes containing x by the
tridiagonal x pass) and on the transform route (two transform pairs instead of three, so the bound
of the 3D Poisson solve applies).  Grids on all three transform variants: matrix cores
(mirror-symmetric axes up to 256 cells), folded half-size and full matrices (seeded
random widths).  Larger grids (200^3, 45 x 30 x 61), where the dense oracle is out of
reach: whole sampled planes against the oracle's single-plane sparse solve, and the properties
that fix an orthogonal projection onto the subspace at any size -- its output lies in
the subspace (plane divergence, dropped component and walls), it keeps the subspace
(curls of random potentials), it is self-adjoint in the face-volume inner product and
idempotent -- and the potential's curl gives the output back.
"""
import numpy as np
import pytest

import synth
from oracle import planes
from oracle.fv import divergence, zero_walls
from oracle.grid import Grid

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


def ctx_kind(nx, ny, nz, kind):
    import paper_1704_08521_amd as lk
    print(f"[case] planes {nx}x{ny}x{nz} {kind}", flush=True)
    c = lk.Context(nx, ny, nz)
    c.set_stretching(kind, 10.0)
    return c, Grid.make(nx, ny, nz, kind=kind)


def ctx_faces(dims, sym):
    import paper_1704_08521_amd as lk
    print(f"[case] planes {dims} symmetric axes {sym}", flush=True)
    faces = [np.linspace(0.0, 1.0, n + 1) if s else asym_faces(n, 60 + a) for a, (n, s) in enumerate(zip(dims, sym))]
    c = lk.Context(*dims)
    c.set_grid(*faces)
    return c, Grid(*faces)


SMALL = [((8, 8, 8), "uniform"), ((12, 10, 8), "tanh"), ((9, 7, 6), "sine"), ((2, 3, 2), "uniform")]
ASYM = [((7, 8, 9), (False, False, False)), ((12, 9, 10), (True, False, True))]


def check_against_oracle(c, g, which, seed):
    b = synth.random_velocity(g.nx, g.ny, g.nz, seed)
    out, psi = c.plane_project(dev(b), which)
    ref, _ = planes.project_plane(g, b, which)
    out = host(out)
    assert rel(out, ref) < 1e-11
    u, v, w = g.unpack(out)
    for comp, k in zip((u, v, w), planes.KEEP[which]):
        if not k:
            assert np.all(comp == 0.0)
    assert np.all(out[g.wall_mask()] == 0.0)
    ref_psi = planes.potential(g, ref, which)
    assert rel(host(psi).reshape(ref_psi.shape), ref_psi) < 1e-11


@pytest.mark.parametrize("which", [1, 2, 3])
@pytest.mark.parametrize("case", SMALL)
def test_plane_projection_matches_oracle(case, which):
    dims, kind = case
    c, g = ctx_kind(*dims, kind)
    check_against_oracle(c, g, which, 70 + which)


@pytest.mark.parametrize("which", [1, 2, 3])
@pytest.mark.parametrize("case", ASYM)
def test_plane_projection_asymmetric_grids(case, which):
    dims, sym = case
    c, g = ctx_faces(dims, sym)
    check_against_oracle(c, g, which, 80 + which)


@pytest.mark.parametrize("which", [1, 3])
@pytest.mark.parametrize("case", [SMALL[1], SMALL[2]])
def test_plane_projection_transform_route(case, which):
    # the planes containing x solve by the tridiagonal x pass on the default (TPT) route;
    # with the TPF route selected they use the x transforms instead
    dims, kind = case
    c, g = ctx_kind(*dims, kind)
    c.set_poisson_method("tpf")
    check_against_oracle(c, g, which, 75 + which)


@pytest.mark.parametrize("which", [1, 3])
def test_plane_projection_transform_route_asymmetric(which):
    c, g = ctx_faces(*ASYM[1])
    c.set_poisson_method("tpf")
    check_against_oracle(c, g, which, 85 + which)


def interior_potential(g, which, rng):
    shape = planes.potential(g, np.zeros(g.nvel()), which).shape
    psi = rng.standard_normal(shape)
    if which == 1:
        psi[:, :, 0] = psi[:, :, -1] = 0.0
        psi[0] = psi[-1] = 0.0
    elif which == 2:
        psi[:, 0] = psi[:, -1] = 0.0
        psi[0] = psi[-1] = 0.0
    else:
        psi[:, :, 0] = psi[:, :, -1] = 0.0
        psi[:, 0] = psi[:, -1] = 0.0
    return psi


def mdot(M, a, b):
    return float(np.dot(M * a, b))


@pytest.mark.parametrize("which", [1, 2, 3])
@pytest.mark.parametrize("case", [((64, 64, 64), "tanh"), ((200, 200, 200), "tanh"), ((45, 30, 61), "sine")])
def test_plane_projection_properties_at_size(case, which):
    dims, kind = case
    c, g = ctx_kind(*dims, kind)
    M = g.pack(*g.face_volumes())
    rng = np.random.default_rng(90 + which)
    x = synth.random_velocity(*dims, 91)
    y = synth.random_velocity(*dims, 92)
    px_t, psi = c.plane_project(dev(x), which)
    px = host(px_t)
    # in the subspace: dropped component and walls zero, plane divergence zero
    u, v, w = g.unpack(px)
    for comp, k in zip((u, v, w), planes.KEEP[which]):
        if not k:
            assert np.all(comp == 0.0)
    assert np.all(px[g.wall_mask()] == 0.0)
    xk = zero_walls(g, planes._mask(g, x, planes.KEEP[which]))
    assert np.max(np.abs(divergence(g, px))) < 1e-10 * np.max(np.abs(divergence(g, xk)))
    # idempotent
    ppx = host(c.plane_project(px_t, which, potential=False)[0])
    assert rel(ppx, px) < 1e-10
    # self-adjoint in the face-volume inner product
    py = host(c.plane_project(dev(y), which, potential=False)[0])
    lhs, rhs = mdot(M, px, y), mdot(M, x, py)
    assert abs(lhs - rhs) < 1e-10 * np.sqrt(mdot(M, x, x) * mdot(M, y, y))
    # keeps the subspace: curls of random potentials vanishing on the walls
    a = planes.curl_of_potential(g, interior_potential(g, which, rng), which)
    pa = host(c.plane_project(dev(a), which, potential=False)[0])
    assert rel(pa, a) < 1e-10
    # the potential vanishes on the walls and its curl gives the projection back
    shape = planes.potential(g, np.zeros(g.nvel()), which).shape
    ps = host(psi).reshape(shape)
    back = planes.curl_of_potential(g, ps, which)
    assert rel(back, px) < 1e-10
    if which == 1:
        walls = [ps[0], ps[-1], ps[:, :, 0], ps[:, :, -1]]
    elif which == 2:
        walls = [ps[0], ps[-1], ps[:, 0], ps[:, -1]]
    else:
        walls = [ps[:, 0], ps[:, -1], ps[:, :, 0], ps[:, :, -1]]
    for wall in walls:
        assert np.max(np.abs(wall)) < 1e-10 * np.abs(ps).max()


@pytest.mark.parametrize("case", [((200, 200, 200), "tanh"), ((45, 30, 61), "sine")])
def test_plane_projection_sampled_planes_at_size(case):
    # whole planes against the oracle's single-plane sparse solve, at sizes the dense
    # oracle cannot reach: the first, a middle and the last plane of each family
    dims, kind = case
    c, g = ctx_kind(*dims, kind)
    b = synth.random_velocity(*dims, 93)
    bd = dev(b)
    for which in (1, 2, 3):
        out, psi = c.plane_project(bd, which)
        u, v, w = g.unpack(host(out))
        shape = planes.potential(g, np.zeros(g.nvel()), which).shape
        ps = host(psi).reshape(shape)
        n = {1: g.ny, 2: g.nx, 3: g.nz}[which]
        for idx in (0, n // 2 + 1, n - 1):
            print(f"[plane] family {which} index {idx}", flush=True)
            ref = planes.project_one_plane(g, b, which, idx)
            if which == 1:
                got = (u[:, idx, :], w[:, idx, :], ps[:, idx, :])
            elif which == 2:
                got = (v[:, :, idx], w[:, :, idx], ps[:, :, idx])
            else:
                got = (u[idx], v[idx], ps[idx])
            for a, r in zip(got, ref):
                assert rel(a, r) < 1e-10


@pytest.mark.parametrize("which", [1, 2, 3])
def test_plane_projection_of_zero_and_of_a_plane_gradient(which):
    # degenerate inputs: zero gives exactly zero; a field whose kept components are a
    # plane gradient (phi varying in all three directions) projects to zero
    c, g = ctx_kind(17, 9, 12, "tanh")
    out, psi = c.plane_project(dev(np.zeros(g.nvel())), which)
    assert not np.any(host(out)) and not np.any(host(psi))
    from oracle.fv import gradient
    phi = synth.random_cells(17, 9, 12, 5)
    gr = gradient(g, phi)
    pg = host(c.plane_project(dev(gr), which, potential=False)[0])
    assert np.max(np.abs(pg)) < 1e-11 * np.max(np.abs(gr))


def test_plane_projection_rejects_bad_arguments():
    from paper_1704_08521_amd import LidKrylovError
    c, g = ctx_kind(6, 5, 4, "uniform")
    v = dev(synth.random_velocity(6, 5, 4, 1))
    with pytest.raises(ValueError):
        c.plane_project(v, 4)
    with pytest.raises(LidKrylovError):  # unknown family, checked by the library itself
        c._check(c.lib.lc_plane_project(c._h, c._ptr(v, c.nvel, "v"), 0, c._ptr(c.vel(), c.nvel, "out"), None))
    with pytest.raises(LidKrylovError):  # out aliasing the input
        c._check(c.lib.lc_plane_project(c._h, c._ptr(v, c.nvel, "v"), 1, c._ptr(v, c.nvel, "out"), None))
