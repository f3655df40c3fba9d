"""Plain, slow FP64 CPU oracle for the SIPG Laplace operator and its hybrid
multigrid solver (Fehn, Munch, Wall, Kronbichler, "Hybrid multigrid methods
for high-order discontinuous Galerkin discretizations", arXiv:1910.01900).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
calls this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, tables
or constants with the HIP library; both sides receive the same seeded inputs.

Every function states the passage of the paper it follows.  The operator is
written as its plain definition (dense basis tabulations, explicit sparse
assembly), with no sum factorization, so that a reader can compare it with
the weak form by eye.

Modules
  basis     1-D GLL/Gauss nodes, Lagrange values and derivatives (Sec. 2)
  mesh      structured box meshes, cubic (Q3) manifold mapping, geometry
  sipg      penalty, assembled SIPG matrix, element-wise apply, diagonal, RHS
  fe        continuous Q_k space with strongly imposed Dirichlet constraints
  transfer  explicit p-, h- and c-transfer matrices (Sec. 3.2)
  solver    Chebyshev smoother, lambda_max, V-cycle, PCG (Alg. 1-3)
  rng       SplitMix64 counter-based generator for the lambda_max start vector

Readings of passages where the paper is silent are listed in the module that
applies them.  Parity status: every function is pinned by the CPU tests in
``tests/test_oracle_*.py`` except the numerical values of the curvilinear
operator, which no external value pins (parity unpinned beyond the
invariants: symmetry, definiteness, Neumann null space, affine limit,
convergence order).
"""
