"""Divergence-free projection and the Krylov vector of eqs. 8-10 (Section 3).

The next Krylov vector (v', p') of a current vector v satisfies eq. 8
(v' = -grad p' + w, w the right side of eq. 10) and eq. 9 (div v' = 0 with the
homogeneous boundary conditions).  It is the projection of w onto the
divergence-free subspace: v' = w - G phi with (D G) phi = D w, p' = phi.

On the staggered grid the homogeneous conditions are carried by the stencil
(tangential wall values) and by the wall-normal faces, which the projection
never changes (G is zero there); step 3 of the paper's loop therefore only
re-zeroes those faces, and with an exact Poisson solve the loop ends after its
first pass.  ``simple_loop`` performs the paper's steps literally to show that.
"""
from __future__ import annotations

import numpy as np

from .fv import divergence, gradient, jacobian_apply, zero_walls
from .grid import Grid
from .poisson import PoissonFD


def vnorm(g: Grid, r):
    """Volume-weighted L2 norm of a cell field, sqrt(sum V r^2)."""
    return float(np.sqrt(np.sum(g.volumes() * np.asarray(r) ** 2)))


class Projector:
    def __init__(self, g: Grid):
        self.g = g
        self.fd = PoissonFD(g)

    def project(self, w):
        """(P w, phi): P w = w - G phi, (D G) phi = D w, sum V phi = 0."""
        g = self.g
        w = zero_walls(g, w)
        phi = self.fd.solve(divergence(g, w))
        return w - gradient(g, phi), phi

    def krylov_vector(self, U, v, re: float):
        """(v', p') = (P L_U v, phi) -- the Krylov vector of eqs. 8-10."""
        return self.project(jacobian_apply(self.g, U, v, re))

    def simple_loop(self, w, eps=1e-13, max_iter=10):
        """The paper's loop: v = w, p = 0; repeat {solve Lap phi = div v with
        Neumann walls; v -= grad phi; p += phi; restore the boundary values}
        until ||phi|| < eps.  Returns (v, p, iterations)."""
        g = self.g
        v = zero_walls(g, w)
        p = np.zeros(g.shapes()[3])
        scale = max(vnorm(g, divergence(g, v)), 1e-300)
        for it in range(1, max_iter + 1):
            phi = self.fd.solve(divergence(g, v))
            v = zero_walls(g, v - gradient(g, phi))
            p = p + phi
            if vnorm(g, phi) <= eps * scale or vnorm(g, divergence(g, v)) <= eps * scale:
                return v, p, it
        return v, p, max_iter


def div_certificate(g: Grid, vec):
    """Scale-free divergence: max_c |sum of signed face fluxes| / max_c sum |fluxes|."""
    u, v, w = g.unpack(vec)
    X, Y, Z = g.X, g.Y, g.Z
    ax = Y.d[None, :, None] * Z.d[:, None, None]
    ay = X.d[None, None, :] * Z.d[:, None, None]
    az = X.d[None, None, :] * Y.d[None, :, None]
    net = (np.diff(u, axis=2) * ax + np.diff(v, axis=1) * ay + np.diff(w, axis=0) * az)
    tot = ((np.abs(u[:, :, 1:]) + np.abs(u[:, :, :-1])) * ax
           + (np.abs(v[:, 1:, :]) + np.abs(v[:, :-1, :])) * ay
           + (np.abs(w[1:]) + np.abs(w[:-1])) * az)
    return float(np.max(np.abs(net)) / max(np.max(tot), 1e-300))
