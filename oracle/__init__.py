"""CPU oracle for the N^5 excited-state-specific MP2 hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP library:
the only common input is the seeded generator in ``synth``.

Two tiers, both plain FP64:

* ``explicit`` -- the definition written out.  Slater determinants as bit
  strings, the Hamiltonian and the Fock operator applied as second-quantised
  operators, the modified zeroth-order Hamiltonian built as an explicit
  matrix on doubles + L-triples, and a direct solve.  Tiny sizes only.
* ``structured`` -- the same operator in the spin-adapted seven-box amplitude
  layout, applied with dense tensor contractions (numpy).  It is pinned to
  ``explicit`` by brute force and runs at every workload size.

``topbasis`` rotates the input to the transition-orbital-pair (TOP) basis,
``layout`` maps the seven-box layout to determinants, ``frontend`` builds
the Fock operator of the reference's density from the one-electron operator
and ``gradient`` differentiates E2 with respect to the TOP-basis Fock matrix
and factor (stationary functional at fixed amplitudes, exact central
differences).
"""
