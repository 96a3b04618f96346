"""Plain, slow FP64 CPU oracle of the meshless FDTD hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
CPU-baseline leg of the benchmark may import or call anything in this
package; the GPU library never routes through it and shares no code with it.
The only module both sides use is ``synth`` (seeded input generators, none of
the method's arithmetic).

What is computed, following Kolar-Pozun & Kosec, "An RBF-based method for
computational electromagnetics with reduced numerical dispersion":

* ``reorder`` -- Morton node order (bit-interleaved quantised coordinates) and
  Reverse Cuthill-McKee on the stencil graph; node order is not part of the
  paper, it only relabels nodes.
* ``knn``     -- stencils: the n nearest nodes of each centre (Section 4.1,
  eq. 11), ordered by (squared distance, original index); brute force.
* ``weights`` -- local PHS + monomial systems (eq. 8-9) solved for RBF-FD
  weights (eq. 13), RBF-VFD weights (eq. 14-15) and the hyperviscosity
  operator (Section 5.1, RBF-FD with phi = r^(2 alpha + 1), m = 2 alpha).
* ``step``    -- the stabilised interleaved leapfrog (eq. 19, with its 3D
  curl generalisation), the energy of eq. 20, the errors of eq. 23, the
  K-field batch and the discrete adjoint of the update.

Every floating-point result is FP64.  Pins (closed forms, invariants, brute
force) live in tests/test_oracle_*.py.
"""
