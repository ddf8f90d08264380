"""Plain FP64 CPU oracle for 4D staggered/HISQ Kahler-Dirac multigrid
(Ayyar, Brower, Clark, Wagner, Weinberg, "Optimizing Staggered Multigrid for
Exascale performance", Lattice 2022, arXiv:2212.12559).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only tests/, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library; both sides take
their inputs from paper_2212_12559_amd.latgen (which holds no arithmetic of
the method).

Every function is the plain definition (or the algorithm's steps in the
paper's order) written in numpy, complex128, with no blocking or fusion.

Every function is pinned by tests/test_oracle_*.py against closed forms,
dense solves, brute force or invariants (the CGNE near-null iteration by its
null-space limit and its Krylov-minimiser property on dense matrices).
"""
from . import operators, solvers  # noqa: F401
