"""Plain, slow, CPU FP64 oracle for commute-time anomaly detection.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library never links, loads
or calls anything here, and nothing here imports the GPU package: the two
share only the seeded input generators (package ``gen``), which hold none of
the method's arithmetic.

What it computes (each function cites the passage it follows):

* graph: squared distances by direct differences, kernel bandwidth, Gaussian
  kernel weights, degrees, volume, Laplacian;
* right-hand sides of Algorithm 1 with counter-based SplitMix64 signs;
* the embedding Z = L^+ Y directly (dense Cholesky, or eigendecomposition);
* commute times (eq. 1 and the embedding form), node anomaly scores
  (Algorithm 4) and the top-K set;
* the inverse chain of Algorithm 2 (normalised, deflated levels and their
  application) and its Richardson iteration, for checking intermediate GPU
  results.

Parity pins (closed forms, invariants, brute force, library routines) live in
``tests/test_oracle_*.py``.  Every function is pinned; none is "parity
unpinned".
"""

from .cad import *  # noqa: F401,F403
