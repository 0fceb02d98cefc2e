"""Newton steady state with a sparse direct saddle-point solve (Section 3, steps 1-4).

F(U) = P R(U) (residual of eqs. 1-4 projected onto the divergence-free space).
The Newton correction d solves the Jacobian system of step 3,

    [ L_U   -G' ] [ d ]   [ R(U) + f ]
    [ D'     0  ] [ q ] = [    0     ]

on interior faces, with one pressure value pinned (G' and D' drop the first
pressure column / continuity row, whose equation is implied by the others), and
U <- U - d (step 4).  ``f`` is an optional body force used for manufactured
solutions.  The sparse matrices are assembled column by column from the
matrix-free operators by probing with colored unit vectors: every stencil
reaches at most one index away along each axis, so inputs three apart never
touch the same output.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fv import divergence, gradient, jacobian_apply, residual, zero_walls
from .grid import Grid
from .simple import Projector


def _layout(shapes):
    """Per-DOF (component, k, j, i) for a list of 3D shapes packed in order."""
    comp, K, J, I, offs = [], [], [], [], []
    off = 0
    for c, s in enumerate(shapes):
        k, j, i = np.meshgrid(np.arange(s[0]), np.arange(s[1]), np.arange(s[2]), indexing="ij")
        comp.append(np.full(k.size, c)); K.append(k.ravel()); J.append(j.ravel()); I.append(i.ravel())
        offs.append(off)
        off += k.size
    return (np.concatenate(comp), np.concatenate(K), np.concatenate(J), np.concatenate(I), offs)


def assemble(apply, in_shapes, out_shapes, in_active=None):
    """Sparse matrix of a linear map whose outputs depend only on inputs at most
    one index away along each axis."""
    cin, kin, jin, iin, offs = _layout(in_shapes)
    cout, kout, jout, iout, _ = _layout(out_shapes)
    nin, nout = cin.size, cout.size
    active = np.ones(nin, bool) if in_active is None else in_active
    rows, cols, vals = [], [], []
    for c, s in enumerate(in_shapes):
        for ck in range(3):
            for cj in range(3):
                for ci in range(3):
                    sel = active & (cin == c) & (kin % 3 == ck) & (jin % 3 == cj) & (iin % 3 == ci)
                    if not sel.any():
                        continue
                    x = np.zeros(nin)
                    x[sel] = 1.0
                    y = apply(x)
                    r = np.nonzero(y)[0]
                    # the unique input index of this color in the window {o-1, o, o+1}
                    kk = kout[r] - 1 + ((ck - (kout[r] - 1)) % 3)
                    jj = jout[r] - 1 + ((cj - (jout[r] - 1)) % 3)
                    ii = iout[r] - 1 + ((ci - (iout[r] - 1)) % 3)
                    ok = ((kk >= 0) & (kk < s[0]) & (jj >= 0) & (jj < s[1]) & (ii >= 0) & (ii < s[2]))
                    col = offs[c] + (kk * s[1] + jj) * s[2] + ii
                    col = np.where(ok, col, 0)
                    ok &= sel[col]
                    if not np.all(ok):
                        raise RuntimeError("stencil wider than one index")
                    rows.append(r); cols.append(col); vals.append(y[r])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nout, nin))


def operator_matrices(g: Grid, U, re: float):
    """(L, G, D, interior index) with L = L_U on all faces (rows/cols), G cells ->
    faces, D faces -> cells."""
    vs = list(g.shapes()[:3])
    ps = [g.shapes()[3]]
    interior = ~g.wall_mask()
    L = assemble(lambda x: jacobian_apply(g, U, x, re), vs, vs, interior)
    G = assemble(lambda q: gradient(g, q.reshape(ps[0])), ps, vs)
    D = assemble(lambda x: divergence(g, x).ravel(), vs, ps, interior)
    return L, G, D, np.nonzero(interior)[0]


def saddle_matrix(g: Grid, U, re: float):
    """The pinned saddle-point matrix [[L, -G'], [D', 0]] on interior faces."""
    L, G, D, it = operator_matrices(g, U, re)
    Li = L[it][:, it]
    Gi = G[it][:, 1:]
    Di = D[1:][:, it]
    A = sp.bmat([[Li, -Gi], [Di, None]], format="csc")
    return A, it


class Newton:
    def __init__(self, g: Grid, re: float, alpha: float, forcing=None):
        self.g, self.re, self.alpha = g, re, alpha
        self.forcing = None if forcing is None else zero_walls(g, forcing)
        self.proj = Projector(g)

    def full_residual(self, U):
        r = residual(self.g, U, self.re, self.alpha)
        return r if self.forcing is None else r + self.forcing

    def F(self, U):
        """(P R(U), pressure) -- the projected residual and its pressure."""
        return self.proj.project(self.full_residual(U))

    def step(self, U):
        """One Newton step; returns (U_new, |F(U)|_inf, |d|_inf)."""
        g = self.g
        U = zero_walls(g, U)
        Fv, _ = self.F(U)
        A, it = saddle_matrix(g, U, self.re)
        rhs = np.zeros(A.shape[0])
        rhs[:it.size] = self.full_residual(U)[it]
        sol = spla.spsolve(A, rhs)
        d = np.zeros(g.nvel())
        d[it] = sol[:it.size]
        return U - d, float(np.max(np.abs(Fv))), float(np.max(np.abs(d)))

    def solve(self, U0=None, tol=1e-10, max_steps=20):
        """Newton iterations until |F|_inf <= tol; returns (U, history of |F|_inf)."""
        U = np.zeros(self.g.nvel()) if U0 is None else zero_walls(self.g, U0)
        hist = []
        for _ in range(max_steps):
            Fv, _ = self.F(U)
            f = float(np.max(np.abs(Fv)))
            hist.append(f)
            if f <= tol:
                break
            U, _, _ = self.step(U)
        return U, hist
