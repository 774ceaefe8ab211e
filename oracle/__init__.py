"""CPU FP64 oracle for the batched BDF astrochemistry solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package; only the tests, the smoke check of the package entry file and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
path: its only input is the seeded synthetic data from ``synth``.

Modules
-------
chem    rate coefficients (paper Sec. 2 Kooij-Arrhenius and cosmic-ray forms,
        App. B.1 photo form), the mass-action right-hand side (paper Sec. 2,
        the rate equation for dn_i/dt) and its analytic Jacobian.
bdf     variable-order, variable-step BDF (quasi-constant step size,
        backward-difference form) for one cell, with frozen-sequence replay and
        discrete forward sensitivities.
esdirk  Kvaerno's seven-stage 5(4) ESDIRK (the paper's integrator, Sec. 4)
        for one cell, on the same Newton iteration as bdf.
steady  steady state of the rate equations by damped Newton with the
        conservation laws substituted for dependent rows.
brute   fixed-step 3-stage Radau IIA reference integrator with step halving.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
closed forms, invariants, library routines or brute force; see the pin table
in the design notes.  The FP32-LU error statement has no pin of its own
("parity unpinned" beyond the stated tolerance).
"""
