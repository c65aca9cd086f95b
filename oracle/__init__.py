"""Plain FP64 CPU oracle for the multi-patch IgA multigrid method of
Takacs, "Fast multigrid solvers for conforming and non-conforming multi-patch
Isogeometric Analysis" (arXiv:1902.01818).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP library; the two meet
only through the seeded input generators in ``workloads``.

Every routine is written for readability, not speed: numpy / scipy sparse
matrices, Gauss quadrature written out, the multigrid cycle as the paper's
recursion.  Each function names the section / equation / algorithm it follows.

Functions without an independent pin say "parity unpinned" in their docstring.
At present every function is pinned by a test under ``tests/oracle``.
"""

from .solver import OracleProblem, setup  # noqa: F401
