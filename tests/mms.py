"""Analytic fields for manufactured-solution checks.

Derivatives are taken from the analytic expressions by 6th-order central
differences with a tiny step (error ~1e-11), far below the O(h^2) discretization
errors being measured, so no derivative is typed by hand.
"""
import numpy as np

PI = np.pi
_H = 2e-3
_C = np.array([-1.0, 9.0, -45.0, 0.0, 45.0, -9.0, 1.0]) / 60.0


def d(f, axis, x, y, z):
    """d f / d(x|y|z) of a scalar function f(x, y, z) at arrays x, y, z."""
    out = 0.0
    for m, c in zip(range(-3, 4), _C):
        if c == 0.0:
            continue
        dx = [0.0, 0.0, 0.0]
        dx[axis] = m * _H
        out = out + c * f(x + dx[0], y + dx[1], z + dx[2])
    return out / _H


def d2(f, axis, x, y, z):
    return d(lambda a, b, c: d(f, axis, a, b, c), axis, x, y, z)


def face_points(g, comp):
    """Coordinates (x, y, z) of the u (0), v (1) or w (2) unknowns, arrays [k, j, i]."""
    xs = [g.X.c, g.Y.c, g.Z.c]
    xs[comp] = (g.X.xf, g.Y.xf, g.Z.xf)[comp]
    z, y, x = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return x, y, z


def cell_points(g):
    z, y, x = np.meshgrid(g.Z.c, g.Y.c, g.X.c, indexing="ij")
    return x, y, z


def sample(g, fields):
    """Pack three scalar functions sampled at the u, v, w points."""
    return g.pack(*[fields[c](*face_points(g, c)) for c in range(3)])


def psi_velocity():
    """u = curl(psi, psi, psi), psi = G(x) G(y) G(z), G(s) = s^2 (1-s)^2:
    divergence-free and zero on every wall (no slip)."""
    def G(s):
        return s * s * (1 - s) ** 2

    def psi(x, y, z):
        return G(x) * G(y) * G(z)

    u = lambda x, y, z: d(psi, 1, x, y, z) - d(psi, 2, x, y, z)
    v = lambda x, y, z: d(psi, 2, x, y, z) - d(psi, 0, x, y, z)
    w = lambda x, y, z: d(psi, 0, x, y, z) - d(psi, 1, x, y, z)
    return [u, v, w]


def wall_normal_free_fields(shift=0.0):
    """Smooth field whose normal component vanishes on every wall."""
    u = lambda x, y, z: np.sin(PI * x) * np.cos(PI * y + shift) * (1 + z * z)
    v = lambda x, y, z: np.sin(PI * y) * np.cos(1.3 * PI * z) * (1 + 0.5 * x)
    w = lambda x, y, z: np.sin(PI * z) * np.cos(0.7 * PI * x + shift) * (1 - 0.3 * y)
    return [u, v, w]


def cos3(x, y, z):
    return np.cos(PI * x) * np.cos(PI * y) * np.cos(PI * z)
