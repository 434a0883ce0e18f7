"""FP64 CPU oracle for the X-MeshGraphNet processor hot path.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct definition that the HIP library is checked against.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import it; the
library never routes through it and shares no code with it.

Modules
  graph      multi-scale kNN point-cloud graph (Sec. III.B, III.C) -> CSR/CSC
  partition  recursive coordinate bisection + L-hop halo (Sec. III.A)
  model      encoder / processor (Eq. 1-4) / decoder, masked MSE loss,
             hand-written adjoint, gradient aggregation over partitions,
             the bfloat16 weight cast of mixed-precision training
  optim      Adam with global-norm clipping, cosine learning rate (Sec. V.D)

Every function is float64 unless it produces integers.  Where the paper is
silent the reading taken is stated in the function's docstring.

Parity status: every function is pinned by tests under tests/ (brute force,
closed forms, invariants, finite differences); none is "parity unpinned".
"""
