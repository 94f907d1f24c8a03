"""CPU oracle for the pilot-wave (gate-by-gate) exact sampler.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package; only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP engine:
the only common module is ``instances`` (seeded graphs and gate lists, which
hold none of the method's arithmetic).

Everything here is plain and slow on purpose: complex128 state vectors and
density matrices, Algorithm 1 (ideal) and Algorithm 2 (noisy) of the paper
written step by step, a path-sum amplitude by variable elimination for large
qubit counts, the QAOA p=1 closed form and state-vector gradients.

Parity pins (tests under ``tests/`` marked ``not gpu``) tie every function to
something other than itself; see each module's docstring.
"""
