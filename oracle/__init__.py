"""FP64 CPU oracle for the single-layer gCQ/3D-ACA hot path.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
definition that the HIP library is checked against.  Only the test-suite, the
smoke check of the build entry point and the CPU-baseline leg of the benchmark
may import it; the library and its Python binding never do, and the two share
no code (only the seeded input generators in ``synth`` feed both).

All floating point is float64 / complex128.  numpy supplies library primitives
(QR, SVD, Gauss-Legendre nodes, matrix products); everything else is written
out step by step in the order of the paper.

Modules
  quadrature  reference-triangle rules (7-point degree-5 rule, Gauss-Legendre)
  geometry    per-panel tables: area, centroid, longest edge, quadrature points
  entries     Laplace-domain single-layer entries V(s)[i, j] (Sec. 3), three tiers
  tree        cluster tree and block cluster tree (Sec. 4, eq. admissible)
  aca         partially pivoted ACA and QR/SVD recompression (Sec. 4)
  aca3d       3D-ACA over the frequencies (Alg. 1, eq. norm)
  matvec      dense, per-frequency H-matrix and compressed products (eq. product)
  gmres       restarted GMRES with classical Gram-Schmidt twice (solver step)
  mlp         the rank-prediction MLP: forward, backward, Adam
  freqmap     conjugate-symmetry map of the frequency set

Readings of points the paper leaves open are stated in each module's docstring.
Parity pinned for every module (see tests/test_oracle_*.py) except where a
module's docstring says "parity unpinned".
"""
