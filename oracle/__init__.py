"""CPU oracle for the all-at-once Uzawa multigrid (UMG) of the P1-P1 PSPG Stokes
system (Gmeiner, Huber, John, Ruede, Wohlmuth, "A quantitative performance
analysis for Stokes solvers at the extreme scale", arXiv:1511.02134).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of the entry
module and the CPU-baseline leg of the benchmark may import this package.  The
GPU library never calls it and shares no code, table or helper with it.

The oracle is deliberately plain: FP64 throughout, the global mesh assembled
element by element from the bilinear forms of Section 2 (scipy sparse
matrices), Gauss-Seidel by colour classes with sparse row slices, dense direct
coarse solves.  It follows the paper's formulas in the paper's order:

  fem.py     -- uniform refinement, P1 element matrices for a_1, b, c_l, the
                right-hand side f and g_l, transfer operator (Section 2.1)
  umg.py     -- inexact Uzawa smoother (eq. Uzawa_smooth), V-cycle, coarse
                solve, stopping criterion (Sections 3.3-3.6)
  krylov.py  -- velocity multigrid with (FHGS, BHGS) smoothing, block-diagonal
                PMINRES and the Schur-complement CG of Algorithm 1
                (Sections 3.1, 3.2, 3.5)
  rows.py    -- single rows of the system at chosen vertices (full-size checks)
  cost.py    -- operator counts, E_TME and memory models (Sections 4.1, 4.2, 5)
  adjoint.py -- gradients of J = 1/2 ||u - u_obs||^2 with respect to the
                forcing and the per-macro viscosity (not in the paper; the
                discrete adjoint of the same symmetric system)

Readings of the paper that the oracle takes where it is silent or ambiguous
are listed in the module docstrings; parity pins live in tests/.
"""
from .fem import Hierarchy, build_hierarchy  # noqa: F401
from .umg import UMG  # noqa: F401
