"""Oracle: a plain, slow, obviously correct CPU implementation of the method.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute anything in this package. Only the tests, the smoke check and the CPU
baseline leg of the benchmark use it, to check the HIP path against it.

Contents (each function cites the passage of Wittmann, Zeiser, Hager and
Wellein, "Modeling and analyzing performance for highly optimized propagation
steps of the lattice Boltzmann method on sparse lattices", that it follows):

* ``d3q19``  - the D3Q19 velocity set, weights and opposite directions.
* ``dense``  - a full-array FP64 D3Q19 BGK stream-and-collide solver with
               halfway bounce-back and a constant body force (Sect. 2, eq. (1)),
               plus a dependency-cone runner that evaluates single sites of a
               large lattice after a few steps.
* ``tables`` - the sparse-lattice integer tables: lexicographic enumeration
               with blocking factor and Morton enumeration (Sect. 1, Sect. 5.6),
               the 18-entry adjacency list (Sect. 4, loop balance), the
               run-length coded "shifted by one" runs of reduced indirect
               addressing (Sect. 4.1) and their per-wavefront encoding.
* ``model``  - the loop-balance model in bytes per fluid lattice update
               (Sect. 4 and Sect. 4.1) and the Roofline prediction (Sect. 5.2).

The oracle shares no code with the HIP path; the two only consume the same
seeded inputs from ``lbm_inputs``.

Every function here has at least one pin in ``tests/`` that is independent of
the oracle itself (closed forms, exact invariants, the paper's worked channel
example, brute force on tiny inputs).
"""
