"""Plain FP64 CPU oracle for the adaptive multigrid Wilson-Dirac solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library shares
no code with it and never calls it.

Every function follows the paper (Babich et al., "Adaptive multigrid algorithm
for the lattice Wilson-Dirac operator", 2010) step by step in numpy
complex128, with no blocking, fusion or reordering beyond what the paper's
definitions state.  Conventions the paper leaves open (gamma basis, boundary
conditions, site order, QR phase) are fixed in ``oracle.wilson`` and
``oracle.transfer`` and listed with their readings in the design notes.
"""
from . import wilson, transfer, coarse, solvers  # noqa: F401
