"""Plain FP64 CPU oracle for the overlap-operator hot path (arXiv:1106.4964).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path (the C-ABI library and its Python binding) never does, and the oracle
never imports the product path.  Both take their inputs from
``synth_inputs`` (random numbers only).

Modules
  lattice  - site ordering, even-odd index, neighbour tables
  dirac    - chiral gamma basis, Wilson D_w (Sec. II, eq. 1-2), H_w = gamma5 D_w
  sign     - Chebyshev approximation of x^{-1/2} (eq. 4), Clenshaw evaluation
             of Q P(Q^2) (eq. 5, Sec. V), low-mode projection (eq. 6-7),
             overlap D and D(m) (eq. 3, eq. 8)
  dense    - dense-matrix references on tiny lattices (exact sign by eigh)
  solvers  - Lanczos spectral bounds, low-mode eigensolver, CG for D(m)
  ptc      - gauge-equivariant parallel-transport convolution layer

All arithmetic is complex128 / float64 unless a function says otherwise.
Pins for every function live in tests/test_oracle_*.py.
"""
