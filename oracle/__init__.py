"""Plain, slow FP64 CPU oracle for Block Belief Propagation on kagome PEPS.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP
library; the only common module is the seeded input generator in ``synth``,
which holds none of the method's arithmetic.

Contents (each module cites the passages of the thesis it follows):

* ``geometry``    kagome lattice, blocks, faces, leg pairing, sweep orders
                  (Ch. "Block Belief Propagation", Sec. "Defining the Kagome
                  block"; App. "Kagome Block Indexing").
* ``rng``         splitmix64 counter-based random signs for the randomized
                  range finder (Steele, Lea & Flood 2014).
* ``dense``       statevector and exact double-layer contractions, plain BP
                  (Eq. BP:DefiningEquation), dense exact-mode BlockBP
                  (Eq. blockBP:DefiningEquation).
* ``bubble``      boundary-MPS contraction (Sec. "The boundary-MPS method")
                  with truncated SVD splits, canonical moves and log-scale.
* ``blockbp``     BlockBP sweeps (Alg. BlockBP_singleBlock and the finite
                  defining equation) and local expectation values
                  (Eq. res:afm-h:hamiltonian).

Parity status of each function is stated in its docstring.
"""
