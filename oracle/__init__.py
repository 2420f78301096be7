"""Plain FP64 CPU oracle of the semi-structured AMG (SSAMG) method.

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports, links or runs
this package; only the tests, the smoke check and the benchmark's CPU-baseline
leg may.  It shares no code with the HIP path (the seeded input generators in
``workloads`` are the only common module, and they hold no solver arithmetic).

Everything is written from the paper's definitions, in its order and notation,
with scipy sparse products standing in for "a matrix product":

  assemble.py  A = S + U from stencil arrays + inter-part couplings, with
               Dirichlet elimination (Section 2); the finite-volume rule used
               by the synthetic workloads and its adjoint gradient.
  ssamg.py     grid-spacing metric W (Section 3.1), Algorithm 1 (coarsening),
               operator-collapse interpolation (Section 3.2, eq:prolEx with the
               sign reading below), Galerkin A_c = P^T A P (eq:galerkin),
               weighted Jacobi with omega_p (eq:relax0, eq:relax1,
               eq:alpha-beta), V(1,1) cycle and PCG (Section 4 protocol).

Parity status of each function is listed in its docstring; every function is
pinned by a ``-m "not gpu"`` test against closed forms, hand-derived values,
dense direct solves, finite differences or structural invariants.
"""
