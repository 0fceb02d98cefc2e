"""Write the stored expected values under tests/golden/ using the oracle only.

    python tests/golden/make_golden.py

* ``spectrum_8_uniform_re100_a0.txt``: all 833 eigenvalues of the stability
  problem (eq. 7) of the 8^3 uniform cube, Re = 100, lid along x (alpha = 0), at
  the Newton steady state.  Written from the QZ pencil and checked here against
  the two other dense constructions (projected Krylov map, null-space pencil).
* ``leading_16_uniform_re100_a0.txt``: the six leading eigenvalues of the 16^3
  uniform cube, Re = 100, alpha = 0 (the first workload: Newton, then Arnoldi
  for the leading eigenvalues), from ARPACK on the oracle's Krylov map.
* ``critical_16_sine_a45.txt``: the critical Reynolds number and frequency of the
  16^3 cube on the sine-stretched grid of eq. 5 with the lid along the diagonal
  (alpha = 45 deg) (oracle.critical: secant on Re Lambda from Re = 2300 and 2500,
  steady states continued from Re = 500).  On this coarse grid a complex pair crosses
  first (a Hopf crossing, as in the paper's cube, though at a grid-scale frequency).

``python tests/golden/make_golden.py critical`` rewrites the last file only.
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import critical as crit  # noqa: E402
from oracle import eigen  # noqa: E402
from oracle.grid import Grid  # noqa: E402
from oracle.newton import Newton  # noqa: E402


def _write(name, lam, header):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        f.write("# " + header.replace("\n", "\n# ") + "\n# real imag\n")
        for z in lam:
            f.write(f"{z.real:.17e} {z.imag:.17e}\n")
    print("wrote", path)


def main():
    g = Grid.make(8)
    U, hist = Newton(g, 100.0, 0.0).solve(tol=1e-13)
    print("8^3 Newton |F|:", hist)
    lp = eigen.pencil(g, U, 100.0)
    ld, _ = eigen.dense_projected(g, U, 100.0)
    ln = eigen.nullspace(g, U, 100.0)
    assert lp.size == ld.size == ln.size == 833
    for other in (ld, ln):
        assert eigen.match_distance(lp, other) < 1e-9
    _write("spectrum_8_uniform_re100_a0.txt", lp,
           "8^3 uniform cube, Re=100, alpha=0, Newton steady state; all eigenvalues of P L_U on\n"
           "the divergence-free space (eq. 7), from the oracle's QZ pencil, checked against\n"
           "its projected-Krylov-map and null-space constructions; ordered by real part")

    g = Grid.make(16)
    U, hist = Newton(g, 100.0, 0.0).solve(tol=1e-12)
    print("16^3 Newton |F|:", hist)
    lam = eigen.arpack(g, U, 100.0, k=6, ncv=30, tol=1e-13)
    _write("leading_16_uniform_re100_a0.txt", lam,
           "16^3 uniform cube, Re=100, alpha=0, Newton steady state; six leading eigenvalues\n"
           "(largest real part) from ARPACK on the oracle's Krylov-vector map")


def critical():
    g = Grid.make(16, kind="sine")
    alpha = math.radians(45.0)
    U = None
    for re in (500.0, 1000.0, 1500.0, 2000.0, 2300.0):
        U, hist = Newton(g, re, alpha).solve(U, tol=1e-11, max_steps=30)
        print(f"16^3 sine alpha 45 Re {re}: Newton |F| {hist[-1]:.1e} after {len(hist)}", flush=True)
    out = crit.critical_re(g, 2300.0, 2500.0, U, alpha=alpha, re_tol=1e-9, max_evals=14, newton_tol=1e-11)
    assert out["converged"], out
    path = os.path.join(HERE, "critical_16_sine_a45.txt")
    with open(path, "w") as f:
        f.write("# 16^3 cube, sine-stretched grid (eq. 5), lid along the diagonal (alpha = 45 deg):\n"
                "# critical Reynolds number and frequency from oracle.critical (secant on Re Lambda\n"
                "# from Re = 2300, 2500; Newton steady states continued from Re = 500 through 1000,\n"
                "# 1500, 2000)\n")
        f.write(f"re_cr {out['re_cr']:.12f}\nomega_cr {out['omega_cr']:.12f}\n")
        f.write("# evaluations: Re, Re Lambda, Im Lambda\n")
        for re, lr, li in out["history"]:
            f.write(f"# {re:.10f} {lr:+.12e} {li:+.12e}\n")
    print("wrote", path, out["re_cr"], out["omega_cr"], flush=True)


if __name__ == "__main__":
    if sys.argv[1:] == ["critical"]:
        critical()
    else:
        main()
        critical()
