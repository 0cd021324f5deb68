"""Oracle: a plain, slow, serial FP64 CPU implementation of the method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The GPU library
(``paper_2311_08757_amd``) neither imports it nor shares any code with it;
both read their inputs from the seeded generators in ``workloads``.

What it computes (paper: Theisen & Stamm, arXiv 2311.08757):
  * fem       -- Q1 discretisation of -Laplace + V (§2, eq:discrete-weak-form),
                 two independent assembly routes;
  * cell      -- the periodic cell problem giving the shift sigma and psi
                 (eq:cell-problem, eq:weak-form-cell-problem);
  * dd        -- overlapping decomposition, partitions of unity, the PerFact
                 coarse space and the one/two-level additive Schwarz
                 preconditioners (§2.2, eq:dd-preconditioners,
                 eq:two-level-preconditioners, §2.3
                 def:algebraic-perfact-coarse-space, §4.1.2 distance PU);
  * pcg       -- preconditioned conjugate gradients (§3, eq:cg-energy-norm-error-reduction);
  * ipm       -- sigma-shifted inverse iteration with B-normalisation (§2),
                 with an exact direct solver or with PCG inner solves;
  * grad      -- derivatives of lambda, sigma and a shifted solve with respect
                 to the potential's parameters (beyond the paper);
  * lopcg     -- inexact SI-preconditioned LOPCG (alg:si-lopcg) and its inner
                 variants of §4.3;
  * ras       -- restricted additive Schwarz (eq:dd-preconditioners,
                 eq:two-level-preconditioners), the stationary RAS iteration
                 (eq:stationary-ras, eq:two-level-stationary-ras-mult-cc) and
                 right-preconditioned GMRES (§3).
"""
