"""FP64 CPU oracle for the finite-element physics path (TEST INFRASTRUCTURE).

This package is the slow, plainly written reference that the device path is
judged against.  Only the test-suite, the smoke check and the benchmark's CPU
baseline may import it; the library and its Python binding never do, and it
imports nothing from them.

Contents
--------
fe      P1 kinematics, linear-elastic and Neo-Hookean constitutive laws,
        element energies / forces / tangents and their global assembly.
prep    Mesh preprocessing that the device path must reproduce bit-exactly:
        reverse Cuthill-McKee numbering, element order, element colouring,
        free-DOF map.
solve   Reduced systems, Jacobi-PCG, direct solves and Newton with load steps.

Every function cites the passage of the paper (arXiv 2601.03086) it follows.
Where the paper is silent the reading used is stated in the docstring.

Parity pinning: every function here is pinned by a test in
``tests/test_oracle_pins.py`` (patch tests, closed-form bar, rigid-body
invariants, symmetry and definiteness, the Neo-Hookean small-strain limit,
finite differences, direct-vs-iterative solves, published hash vectors).
"""
