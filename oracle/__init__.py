"""Plain FP64 CPU oracle for SIMPLE-evaluated Krylov vectors of the lid-driven cube.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call, link or
execute anything under ``oracle/``; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library.

What it computes (Gelfgat, "Linear instability of the lid-driven flow in a cubic
cavity"):

* ``grid``    -- face coordinates (uniform, the sine stretching of Section 3
                 eq. 5, and a tanh stretching) and the finite-volume metrics.
* ``fv``      -- the staggered finite-volume operators: divergence, gradient,
                 Laplacian with the lid condition (eqs. 3-4), conservative
                 convection, the momentum residual and its exact Jacobian
                 (the linearized momentum of eq. 6, right side of eq. 10).
* ``poisson`` -- the Neumann pressure-correction Poisson problem solved exactly
                 by a full tensor-product (fast diagonalization) factorization,
                 the TPF idea of Section 3.
* ``simple``  -- the divergence-free projection, the Krylov vector of
                 eqs. 8-10 and the paper's SIMPLE-like loop (Section 3).
* ``newton``  -- Newton steps (Section 3, steps 1-4) with a sparse direct
                 saddle-point solve.
* ``eigen``   -- leading eigenvalues of eq. 7 by three independent dense
                 constructions and by ARPACK.
* ``nn``      -- direct-loop 3D convolution network used to check the learned
                 pressure-correction guess.

Everything is float64 and written for clarity, not speed.
"""
