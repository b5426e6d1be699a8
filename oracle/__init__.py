"""CPU oracle for the PHSVDS hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, float64 implementation of what the GPU path computes, written
from the paper (Wu & Stathopoulos, "A Preconditioned Hybrid SVD Method for
Computing Accurately Singular Triplets of Large Matrices").  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the product path never calls it and shares no code with it.

Modules
-------
dense     one-sided Jacobi (Hestenes) SVD: the plain definition of the k
          smallest/largest singular triplets on small inputs; triplet
          residuals (the acceptance test of Section 5).
phsvds    the two-stage method: block GD+k on C = A^T A (Section 2.2/2.4,
          Algorithm 1 with the dynamic tolerance of Section 3.1), the
          post-processing Rayleigh-Ritz (Section 3.1), and GD+k with the
          refined projection on B = [0 A^T; A 0] (Algorithm 2).
precond   Jacobi preconditioner, the projected correction equation solved by
          CG (exact corrections), and the message-passing network used as a
          learned preconditioner with its forward/backward pass and Adam.
rng       counter-based SplitMix64 stream for the random vectors the method
          draws (replacement of dependent basis columns, random left vectors).

Parity status of each function is stated in its docstring; functions whose
results are not fixed by the paper or by mathematics say "parity unpinned".
"""
