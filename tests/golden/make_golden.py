"""Write the stored expected values under tests/golden/ using the oracle only.

    python tests/golden/make_golden.py

* ``spectrum_8_uniform_re100_a0.txt``: all 833 eigenvalues of the stability
  problem (eq. 7) of the 8^3 uniform cube, Re = 100, lid along x (alpha = 0), at
  the Newton steady state.  Written from the QZ pencil and checked here against
  the two other dense constructions (projected Krylov map, null-space pencil).
* ``leading_16_uniform_re100_a0.txt``: the six leading eigenvalues of the 16^3
  uniform cube, Re = 100, alpha = 0 (the first workload: Newton, then Arnoldi
  for the leading eigenvalues), from ARPACK on the oracle's Krylov map.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

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


if __name__ == "__main__":
    main()
