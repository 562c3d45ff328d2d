"""FP64 CPU oracle for the deflated, Schwarz-preconditioned GCR solver.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. It shares no code with the HIP
library (paper_0706_2298_amd) and never imports it; the only code the two have
in common is the seeded input generator ``latgen``.

What it follows, in M. Luescher, "Local coherence and deflation of the low
quark modes in lattice QCD":

* ``dirac`` -- the Dirac operator of eq. (3.9), read as the plain Wilson
  operator (csw = 0) with periodic boundaries (section 2.1 names the
  O(a)-improved operator; the clover term is not part of this build);
* ``sap`` -- the Schwarz alternating procedure used as the preconditioner of
  eq. (6.2) and as the relaxation of eq. (5.1), with minimal-residual block
  solves (the paper defers both to its refs.; reading stated in ``sap``);
* ``block_gram_schmidt`` -- block restriction and Gram-Schmidt, eq. (4.2);
* ``restrict`` / ``prolong`` / ``proj_P`` -- the block projector, eq. (4.1);
* ``little_operator`` / ``little_apply`` -- eqs. (3.2) and (A.1);
* ``Deflation.PL`` / ``PR`` / ``coarse`` -- eqs. (3.3), (3.4), (3.10);
* ``gcr`` / ``solve`` -- the flexible GCR of section 6.2 on eq. (6.2), with
  restarts recomputing the residual (appendix A.5) and the final solution of
  eq. (3.10), stopping at ||eta - D psi|| <= tol ||eta|| (section 6.3);
* ``inverse_iteration`` / ``setup`` -- the subspace generation of eq. (5.1);
* ``oracle.net`` -- the start-field network (periodic 3^4 convolutions, SiLU),
  its backward pass, the block deficit loss built on eq. (3.15) with its
  gradient, and the Adam update (the paper has no network; the definitions
  are stated in that module).

Pins (tests/test_oracle_*.py): free-field spectrum and plane waves, the
Clifford algebra, gamma5-hermiticity, gauge covariance, dense LAPACK solves
and eigenvalues, the projector identities (3.5)-(3.8), the Schur inverse
(3.14), the determinant factorisation (6.3), the free-field deficit of
eq. (4.4) in closed form, and the block sparsity of fig. 4; for the network,
a brute-force convolution, finite differences of every forward map, the
deficit through the Gram-Schmidt projector, and Adam's first step.
"""
from .dfl import *  # noqa: F401,F403
from .dfl import __all__  # noqa: F401
