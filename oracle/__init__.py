"""FP64 CPU oracle for the tensor-network contraction path (test infrastructure).

This package is test infrastructure, not product code. Only the test suite,
the smoke entry point and the benchmark's CPU-baseline leg may import it. It is
deliberately plain and slow, computes in complex128, and shares no code with
the HIP path: it builds its own gate matrices, its own superoperator tensors
and its own networks from circuit descriptions.

Routes, each following the passage it cites:
  * statevector  - brute-force 2^N state vector (the plain definition of the
                   circuit's output state; Sec. Introduction, problem statement)
  * tensornet    - folded (superoperator) tensor network contracted pairwise
                   with numpy.tensordot (Sec. Preliminaries, eq. (1) and the
                   superoperator tensors printed there)
  * closed_form  - p=1 QAOA edge expectation <Z_u Z_v> with the triangle term
  * gradients    - central finite differences and the per-gate parameter-shift
                   rule for QAOA <C>

Gate conventions (shared by every route of this package):
  R_P(theta) = exp(-i theta P / 2) for P in {X, Y, Z};  ZZ(theta) =
  exp(-i theta Z(x)Z / 2). A two-qubit gate on (q0, q1) has basis index
  2*x_q0 + x_q1 (q0 is the most significant). The QAOA circuit is
  H^n |0>, then for k = 1..p: exp(-i gamma_k Z_u Z_v) on every edge and
  exp(-i beta_k X) on every qubit, i.e. ZZ(2 gamma_k) and R_X(2 beta_k).
"""
