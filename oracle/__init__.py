"""AMG-DD oracle: a plain, slow, serial FP64 CPU implementation of what the
GPU path computes, written from the paper (Mitchell, Strzodka, Falgout,
"Parallel Performance of Algebraic Multigrid Domain Decomposition").

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library and never calls it.

Modules
  amg        RS hierarchy: strength, first-pass C/F splitting, direct
             interpolation, Galerkin product (Section 2)
  composite  composite sets D_l / Dbar_l and local operators (Sections 3, 4.1-4.2)
  cycles     V-cycle (Algorithm 1), AlgFAC (Algorithm 4), masked full-grid
             cycle (Section 4 guiding principle), AMG-DD (Algorithm 2)
  adjoint    dense adjoint and face gradients (derivative of a linear solve)
  parallel   the AMG-DD iteration with its subdomain loop in worker processes

Parity status: every function is pinned by tests under tests/ (dense solves,
closed-form composite sizes, special-case reductions, invariants) except the
float32 emulation of the mixed-precision form, whose parity is unpinned.
"""
from . import amg, composite, cycles, adjoint, parallel  # noqa: F401
