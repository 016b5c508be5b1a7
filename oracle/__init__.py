"""CPU FP64 oracle for the HDG trace operator and its nested multigrid solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or executes this package; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use
it.  It shares no code, tables or constants with the HIP path.

The oracle follows Fabien, Knepley, Mills, Riviere, "Manycore parallel
computing for a hybridizable discontinuous Galerkin nested multigrid method"
(arXiv:1705.09907).  Every function cites the section / equation / algorithm
it restates.  It is written plainly: explicit local HDG systems (Sec. 3,
eqs. static_1/static_2), static condensation (eq. shur0) substituted into the
transmission condition (eq. shur1), an assembled sparse trace matrix, a sparse
direct solve, and the nested p/h V-cycle (Algs. algo_1/algo_2) step by step.

Modules
  quadrature  1D Gauss-Legendre / Gauss-Lobatto rules, barycentric Lagrange
              evaluation and differentiation (Sec. 4).
  mesh        numbering of elements, interior faces and trace DoFs.
  hdg         local matrices, condensed blocks, global assembly, RHS, direct
              solve, reconstruction and L2 errors (Secs. 3 and 5).
  mg          p-transfers, h-transfers, Galerkin Q1 hierarchy, smoothers and
              the V-cycle / solve driver (Secs. 6 and 7), K-cycle and flexible CG.
  adjoint     misfit of the volume solution and its gradient with respect to
              per-element log-coefficients by the adjoint method (an extension
              built from eqs. shur0 / shur1; pinned by finite differences).

Every function listed here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against values the paper prints, closed forms,
invariants or library routines.  Two results are "parity unpinned":

* the absolute L2 error constants of Sec. 5, Table tab1.  The oracle matches
  the printed convergence RATES (within 0.1 at p = 3..5, N = 8..32) but not the
  printed error VALUES: its ||u - u_h|| is 2.0-2.6 times and its ||q - q_h||
  4.8-6.2 times the printed numbers, the factor growing with p (p = 3, N = 8:
  1.14e-6 and 6.18e-6 against 5.49e-7 and 1.27e-6).  No reading tried closes
  the gap for both columns (tau from 0.25 to 16, K^-1 in place of K, K = 1,
  Gauss-Lobatto collocated element matrices, nodal quadrature in the norms),
  so the values are not used as pins;
* the multigrid convergence factor, which the paper reports only for a
  different smoother (see mg.py).
"""
