"""Critical Reynolds number and Richardson extrapolation (test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg use this package.

Definitions followed (Section 2, eq. 7 and the paragraph after it; Section 5):

* the leading eigenvalue Lambda of the stability problem (eq. 7) is the one with the
  largest real part; the flow is stable while Re Lambda < 0, and the critical Reynolds
  number Re_cr is where Re Lambda crosses zero; the critical frequency is the imaginary
  part of Lambda there;
* Richardson extrapolation to zero grid size from the values on two grids, assuming the
  error is O(h^2) with h = 1/N (Section 5.1 for the 2D problem, Section 5.2 and Table 3
  for the cube).

The paper does not say how the root Re_cr was located.  This oracle uses the secant
method on Re -> Re Lambda(Re); every evaluation is a Newton steady state at that Re
(oracle.newton, sparse direct Jacobian solves), started from the linear extrapolation
of the two previous steady states in Re, followed by ARPACK on the oracle's Krylov map
(oracle.eigen.arpack).  The critical frequency is |Im Lambda| interpolated linearly
in Re between the last two evaluations.  When the search does not meet its tolerance
within max_evals (noise in Re Lambda from imperfect steady states), the reported values
come instead from the linear root between the evaluations closest to zero on either side
of it.
"""
import numpy as np

from . import eigen
from .grid import Grid
from .newton import Newton


def secant_step(re_a, f_a, re_b, f_b):
    """Next iterate of the secant method for the root of f (f_a != f_b)."""
    return re_b - f_b * (re_b - re_a) / (f_b - f_a)


def richardson(n_coarse, v_coarse, n_fine, v_fine, order=2):
    """Extrapolation to h = 0 of a quantity with error c h^order, h = 1/N, from its
    values on an N_coarse and an N_fine grid (Section 5)."""
    hc, hf = 1.0 / n_coarse, 1.0 / n_fine
    return (v_fine * hc ** order - v_coarse * hf ** order) / (hc ** order - hf ** order)


def leading(g: Grid, U, re, k=6, ncv=40):
    """The leading eigenvalue (largest real part; positive imaginary part of a pair)."""
    lam = eigen.arpack(g, U, re, k=k, ncv=ncv, tol=1e-12, maxiter=50000)
    lead = lam[np.argmax(lam.real)]
    return complex(lead.real, abs(lead.imag))


def predict(flows, re):
    """Initial Newton guess at re: linear extrapolation in Re of the last two steady
    states (the last one alone if there is only one)."""
    if len(flows) == 1:
        return flows[-1][1].copy()
    (ra, ua), (rb, ub) = flows[-2], flows[-1]
    return ub + (ub - ua) * ((re - rb) / (rb - ra))


def critical_re(g: Grid, re0, re1, U0, alpha=0.0, re_tol=1e-8, max_evals=12, newton_tol=1e-11,
                leading_fn=None):
    """Secant search for Re_cr from the two starting values re0, re1.

    U0 is a steady state (or a good Newton guess) at re0.  Returns a dict with re_cr,
    omega_cr, converged and the history [(Re, Re Lambda, Im Lambda)].  leading_fn(g, U,
    re) replaces the eigenvalue computation (tests pass a synthetic one)."""
    lead = leading if leading_fn is None else leading_fn
    flows, hist = [], []

    def evaluate(re, guess):
        U, _ = Newton(g, re, alpha).solve(guess, tol=newton_tol, max_steps=30)
        flows.append((re, U))
        lam = lead(g, U, re)
        hist.append((re, lam.real, lam.imag))
        return lam

    evaluate(re0, U0)
    evaluate(re1, predict(flows, re1))
    while len(hist) < max_evals:
        (ra, fa, _), (rb, fb, _) = hist[-2], hist[-1]
        if fb == fa:
            break
        rn = secant_step(ra, fa, rb, fb)
        if abs(rn - rb) <= re_tol * abs(rb):
            (_, _, wa), (_, _, wb) = hist[-2], hist[-1]
            omega = wb + (wb - wa) * (rn - rb) / (rb - ra)
            return {"re_cr": rn, "omega_cr": omega, "converged": True, "history": hist}
        evaluate(rn, predict(flows, rn))
    # not converged (noisy or slow): the linear root between the evaluations closest to
    # zero on either side of it, when both exist; otherwise the last secant iterate
    neg = [h for h in hist if h[1] < 0.0]
    pos = [h for h in hist if h[1] > 0.0]
    if neg and pos:
        (ra, fa, wa), (rb, fb, wb) = max(neg, key=lambda h: h[1]), min(pos, key=lambda h: h[1])
        rn = secant_step(ra, fa, rb, fb)
    else:
        (ra, fa, wa), (rb, fb, wb) = hist[-2], hist[-1]
        rn = secant_step(ra, fa, rb, fb) if fb != fa else rb
    return {"re_cr": rn, "omega_cr": wb + (wb - wa) * (rn - rb) / (rb - ra), "converged": False,
            "history": hist}
