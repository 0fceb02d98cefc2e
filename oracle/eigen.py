"""Leading eigenvalues of the linear stability problem (Section 3, eq. 7).

The eigenproblem J x = lam x on velocity and pressure with the continuity
constraint is the eigenproblem of P L_U on the divergence-free space S (the
pressure is slaved to the velocity through the projection).  Three independent
dense constructions and one Krylov one:

* ``dense_projected``: the matrix of the Krylov-vector map v -> P L_U v built
  column by column on interior unit vectors; its spectrum is that of P L_U on S
  plus (n_cells - 1) exact zeros (the gradient directions, which P maps into S),
  which are dropped.
* ``pencil``: finite generalized eigenvalues of ([[L, -G'], [D', 0]],
  diag(I, 0)) with one pressure pinned (QZ).
* ``nullspace``: with Z an orthonormal basis of null(D), the M_u-weighted
  reduced pencil (Z^T M_u L Z, Z^T M_u Z); no projection and no pressure.
* ``arpack``: ARPACK's implicitly restarted Arnoldi (the paper's ref. [33]),
  largest real part, on the Krylov-vector map with the gradient directions
  shifted far left (see ``arpack``).

Ordering: real part descending; within a complex-conjugate pair the member
with positive imaginary part first.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse.linalg as spla

from .fv import divergence
from .grid import Grid
from .newton import operator_matrices, saddle_matrix
from .simple import Projector


def order(lam):
    lam = np.asarray(lam, dtype=complex)
    key = np.lexsort((-lam.imag, -np.round(lam.real, 12)))
    return lam[key]


def dense_projected(g: Grid, U, re: float):
    proj = Projector(g)
    it = np.nonzero(~g.wall_mask())[0]
    n = g.nvel()
    A = np.empty((it.size, it.size))
    for col, dof in enumerate(it):
        e = np.zeros(n)
        e[dof] = 1.0
        A[:, col] = proj.krylov_vector(U, e, re)[0][it]
    lam = np.linalg.eigvals(A)
    nzero = g.nx * g.ny * g.nz - 1
    keep = np.argsort(np.abs(lam))[nzero:]
    return order(lam[keep]), A


def pencil(g: Grid, U, re: float):
    A, it = saddle_matrix(g, U, re)
    A = A.toarray()
    B = np.zeros_like(A)
    B[np.arange(it.size), np.arange(it.size)] = 1.0
    alpha, beta = scipy.linalg.eig(A, B, right=False, homogeneous_eigvals=True)
    finite = np.abs(beta) > 1e-8 * np.abs(alpha).max()
    return order(alpha[finite] / beta[finite])


def nullspace(g: Grid, U, re: float):
    L, _, D, it = operator_matrices(g, U, re)
    Di = D[:, it].toarray()
    Z = scipy.linalg.null_space(Di)
    mu, mv, mw = g.face_volumes()
    Mu = g.pack(mu, mv, mw)[it]
    Li = L[it][:, it].toarray()
    lam = scipy.linalg.eigvals(Z.T @ (Mu[:, None] * (Li @ Z)), Z.T @ (Mu[:, None] * Z))
    return order(lam)


def shift_bound(g: Grid, U, re: float):
    """A value left of the whole spectrum of L_U (Gershgorin-type bound)."""
    lap = 0.0
    for ax in (g.X, g.Y, g.Z):
        lap += np.max(2.0 / (ax.d * np.minimum(ax.dd[:-1], ax.dd[1:])))
    hmin = min(ax.d.min() for ax in (g.X, g.Y, g.Z))
    return -(1.0 + 2.0 * lap / re + 8.0 * float(np.max(np.abs(U))) / hmin)


def arpack(g: Grid, U, re: float, k: int, ncv: int = 20, tol: float = 1e-12, v0=None,
           return_vectors=False, sigma=None, maxiter=5000):
    """ARPACK, largest real part, on B = P L_U + sigma (I - P).

    B equals P L_U on S and sigma times the identity on the gradient directions
    (block triangular in S + range(G)), so with sigma left of the spectrum the
    wanted eigenvalues are those of P L_U on S, while the zero eigenvalues that
    P L_U has on the gradient directions -- which the restart filter would
    otherwise amplify out of rounding noise -- are moved out of the way.
    """
    proj = Projector(g)
    it = np.nonzero(~g.wall_mask())[0]
    n = g.nvel()
    sig = shift_bound(g, U, re) if sigma is None else sigma

    def mv(x):
        full = np.zeros(n)
        full[it] = np.real(x)
        a = proj.krylov_vector(U, full, re)[0]
        px = proj.project(full)[0]
        return (a + sig * (full - px))[it]

    if v0 is None:
        v0 = np.ones(n)
    v0 = proj.project(np.asarray(v0, float))[0][it]
    op = spla.LinearOperator((it.size, it.size), matvec=mv, dtype=np.float64)
    lam, vec = spla.eigs(op, k=k, which="LR", ncv=ncv, tol=tol, v0=v0, maxiter=maxiter)
    idx = np.lexsort((-lam.imag, -np.round(lam.real, 12)))
    if return_vectors:
        full = np.zeros((n, k), complex)
        full[it] = vec[:, idx]
        return lam[idx], full
    return lam[idx]


def ritz_residual(g: Grid, U, re: float, lam, x):
    """Relative eigen-residual |P L_U x - lam x| / (|lam| |x|) with the oracle's
    own operator (complex x handled by linearity)."""
    proj = Projector(g)
    Ax = proj.krylov_vector(U, x.real, re)[0] + 1j * proj.krylov_vector(U, x.imag, re)[0]
    return float(np.linalg.norm(Ax - lam * x) / (abs(lam) * np.linalg.norm(x)))


def divergence_of(g: Grid, x):
    return divergence(g, x)


def match_distance(a, b):
    """Largest distance from each eigenvalue of ``a`` to its nearest unused
    partner in ``b`` (greedy, in order of ``a``); the spectra must have equal size."""
    a = np.asarray(a, complex)
    b = list(np.asarray(b, complex))
    worst = 0.0
    for z in a:
        k = int(np.argmin([abs(z - y) for y in b]))
        worst = max(worst, abs(z - b.pop(k)))
    return worst
