"""FP64 CPU oracle for the space-time multigrid hot path (test infrastructure only).

This package is the independent reference that the GPU library is checked
against.  It assembles sparse space-time matrices explicitly and solves them
with SciPy, written for clarity rather than speed.  It shares no code with the
GPU path and must only be imported by the tests, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``.

Modules
  basis      1D quadrature rules and Lagrange bases (Section 2, Q_p space; Appendix-style node sets)
  temporal   dG(k) and cGP(k) time matrices and slab-level Kronecker factors
             (Sections 2.1 and 2.2, eqs. dg-time-weights, cg-time-weights)
  spatial    meshes, cell matrices by quadrature, assembled M_h and A_h (eq. space-matrices)
  spacetime  the all-at-once slab operator (eqs. heat-cg-dg-at-once ... wave-cg-cg-at-once)
  rhs        slab right-hand sides and velocity recovery
  mg         transfers, cell-wise additive Schwarz smoother, V-cycle (Section 3, Alg. stmg)
  krylov     flexible GMRES with a V-cycle preconditioner (Section 4 solver setup)
  norms      L2(L2) errors and wave energy
  cnn        FP64 reference of the learned preconditioning stage (not in the paper: parity unpinned)
"""
