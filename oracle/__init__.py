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

Parity status: every function is pinned by a test under tests/ that does
not retype its own formula:
  graph      brute-force kNN, tie lattices, the cross-level dedupe invariant
  partition  backward reachability (scipy), partitioned = full graph at halo L
  model      hand-worked edge features (sign, norm, affine); the whole step
             against float64 torch autograd (both activations, both
             aggregated quantities); closed forms (zero MLPs, the sparse
             adjacency product, LayerNorm statistics); node-permutation
             equivariance; exact translation invariance; central finite
             differences; bfloat16 rounding against torch's conversion
  optim      Adam, clipping and the cosine schedule against torch's CPU ones
No function is "parity unpinned".
"""
