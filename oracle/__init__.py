"""Plain FP64 CPU oracle for synchronous Gaussian belief propagation.

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  The HIP solver never
calls it, links it or shares code with it; the two meet only in the seeded
input generators of ``workloads``.

Everything here follows Bickson, "Gaussian Belief Propagation: Theory and
Application" (arXiv:0811.2518):

* ``dense_solve`` / ``dense_marginal_precisions`` -- the plain definition the
  method reaches: x* = A^-1 b and P_i = 1/(A^-1)_ii (Prop. "linear system ->
  inference", Ch. 2 Sec. 2.1).
* ``naive_gabp`` -- Alg. 1 (Ch. 2, Sec. "The Gaussian BP Algorithm"), scalar
  loops, exact with ``fractions.Fraction`` inputs.
* ``broadcast_gabp`` -- Alg. 2 (Ch. 3, Sec. "GaBP Broadcast Variant"),
  vectorised over the directed edges, synchronous (two message buffers,
  Ch. 2 end of Sec. "The Gaussian BP Algorithm").
* ``aitken_extrapolate`` / ``aitken_gabp`` -- Aitken's extrapolation of the
  means over three successive rounds (Ch. 3 Sec. "Convergence Acceleration").
* ``augmented_csr`` / ``augmented_solution`` -- the symmetric block matrix of
  Ch. 5 Sec. "Extension to General Linear Systems" for a rectangular B, and
  the x-part of its solution by block elimination (the section's lemma).
* ``fixpoint_violation`` -- the message equations of Alg. 2 evaluated on
  converged messages.
* ``is_strictly_dd``, ``walk_rho``, ``rate_bound`` -- the sufficient conditions
  of Ch. 2 Sec. "Convergence and Exactness" and the rate bound of Ch. 3
  Sec. "Upper Bound on Convergence Rate".
* ``convfix_dense`` / ``convfix_gabp`` -- the diagonal-loading double loop of
  Ch. 5 (eq. of Sec. "Iterative Correction Method").
* ``adjoint_gradient`` / ``fd_gradient`` -- dense reference gradients of
  L = 0.5 ||A^-1 b - t||^2 (the solve x = A^-1 b of Prop. 2.1, differentiated).

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""
from .gabp_oracle import *  # noqa: F401,F403
