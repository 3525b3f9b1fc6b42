"""Oracle for the Newton-step KKT solve: TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 CPU implementations of what the library computes, used
to check it. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here; the
library itself never does, and nothing here imports the library.

Contents:
  dense   -- explicit systems (condensed, 2x2 saddle-point, 3x3 augmented),
             Bunch-Kaufman LDL^T with inertia, residual evaluators,
             Schur-complement closed forms.
  sparse  -- ctypes front end to ``sparse_ldl.c``: up-looking sparse LDL^T
             with static pivots (condensed Cholesky, saddle-point LDL^T),
             Richardson refinement and the Cholesky + CG HyKKT solve.
  symbolic -- brute-force boolean elimination (column structures of L).
  ipm     -- primal-dual interior-point method on a convex QP whose Newton
             steps go through the augmented / condensed KKT systems.
"""
