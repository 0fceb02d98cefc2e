"""CPU checks of the benchmark's host-side set-up: the interpolation of a coarse steady
state to the benchmark grid (its result is projected and refined by Newton on the GPU, so
it only has to be a consistent first-order start) and the Richardson extrapolation."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def faces_tanh(n, ratio=10.0):
    beta = np.arccosh(np.sqrt(ratio))
    xi = np.arange(n + 1) / n
    return 0.5 * (1.0 + np.tanh(beta * (2.0 * xi - 1.0)) / np.tanh(beta))


def pack(fx, fy, fz, fu, fv, fw):
    """u|v|w of fields given as functions of (x, y, z) at the staggered positions."""
    c = lambda f: 0.5 * (f[1:] + f[:-1])
    Z, Y, X = np.meshgrid(c(fz), c(fy), fx, indexing="ij")
    u = fu(X, Y, Z)
    Z, Y, X = np.meshgrid(c(fz), fy, c(fx), indexing="ij")
    v = fv(X, Y, Z)
    Z, Y, X = np.meshgrid(fz, c(fy), c(fx), indexing="ij")
    w = fw(X, Y, Z)
    return np.concatenate([u.ravel(), v.ravel(), w.ravel()])


def test_prolongation_reproduces_linear_fields():
    coarse = [faces_tanh(12), faces_tanh(10), faces_tanh(9)]
    fine = [faces_tanh(23), faces_tanh(20), faces_tanh(17)]
    fu = lambda x, y, z: 1.0 + 2.0 * x - 0.5 * y + 0.25 * z
    fv = lambda x, y, z: -x + 3.0 * y + z
    fw = lambda x, y, z: 0.5 + x + y - 2.0 * z
    Uc = pack(*coarse, fu, fv, fw)
    Uf = bench.prolongate_velocity(Uc, coarse, fine)
    ref = pack(*fine, fu, fv, fw)
    assert Uf.shape == ref.shape
    # exact between the coarse positions; clamped (first order) in the half cells next to walls
    c = lambda f: 0.5 * (f[1:] + f[:-1])
    inside = []
    for (fx, fy, fz), (gx, gy, gz) in (((fine[0], c(fine[1]), c(fine[2])), (coarse[0], c(coarse[1]), c(coarse[2]))),
                                       ((c(fine[0]), fine[1], c(fine[2])), (c(coarse[0]), coarse[1], c(coarse[2]))),
                                       ((c(fine[0]), c(fine[1]), fine[2]), (c(coarse[0]), c(coarse[1]), coarse[2]))):
        m = [(a >= b[0]) & (a <= b[-1]) for a, b in ((fz, gz), (fy, gy), (fx, gx))]
        inside.append((m[0][:, None, None] & m[1][None, :, None] & m[2][None, None, :]).ravel())
    inside = np.concatenate(inside)
    assert inside.sum() > 0.5 * inside.size
    assert np.max(np.abs(Uf[inside] - ref[inside])) < 1e-12
    assert np.max(np.abs(Uf - ref)) < 0.5  # near the walls: the nearest coarse value


def test_richardson_matches_paper_tables():
    # Table 3: each extrapolated entry from the current and the previous coarser grid; the
    # printed values look computed from unrounded grid values, hence 0.02 (0.05 for 256^3)
    a0 = [(100, 1963.74, 0.575370), (150, 1938.98, 0.581315), (200, 1930.40, 0.583398), (256, 1926.10, 0.584438)]
    ex0 = [(1919.16, 0.58607), (1919.37, 0.58607), (1919.37, 0.58607)]
    a45 = [(100, 2266.29, 0.250855), (150, 2278.39, 0.250305), (200, 2283.17, 0.249868), (256, 2285.56, 0.249650)]
    ex45 = [(2288.06, 0.24986), (2289.31, 0.249307), (2289.31, 0.249307)]
    for rows, ex in ((a0, ex0), (a45, ex45)):
        for (c, f), (re_x, om_x) in zip(zip(rows, rows[1:]), ex):
            tol = 0.05 if f[0] == 256 else 0.02
            assert abs(bench.richardson(c[1], f[1], c[0], f[0]) - re_x) < tol, (c, f)
            assert abs(bench.richardson(c[2], f[2], c[0], f[0]) - om_x) < 2e-4, (c, f)
