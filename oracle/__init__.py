"""CPU FP64 oracle for the corrector systems of the one-domain
Navier-Stokes-Brinkman solver (Arico, Helmig, Puleo, Schneider,
arXiv 2309.03543).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It is a plain, slow, obviously correct
restatement of what the paper defines, written in NumPy/SciPy in float64,
and shares no code with the GPU library.

Modules
  geometry   per-cell geometry, side pairing, transmissibilities (Sec. 3.2.2,
             eq. cs1_discr; Appendix A side numbering)
  ordering   reverse Cuthill-McKee renumbering and the CSR pattern
  assemble   cell tensors and the CP1 / CP2 matrices (eq. CS1_sys_coeff,
             eq. Cs2_4, eq. CS2_sys_coeff)
  pcg        Jacobi-preconditioned conjugate gradients with residual
             replacement; dense Cholesky reference (Sec. 3.2.2-3.2.3)
  adjoint    adjoint solve and parameter gradients (derived from the
             symmetric corrector systems)
  crossflux  co-normal tangential flux terms of the CP2 and the right-hand
             side B_2 of its second solve (Sec. 3.2.3, eq. Cs2_7,
             eq. eta_flux; App. C, eq. A3.1-A3.2)
  cp1coupled the x/y coupling of the CP1 through the anisotropic mass
             tensor and the paper's loop over the two scalar solves
             (Sec. 3.2.2, eq. cs1_sys2, eq. CS1_sys_coeff; App. B, eq. A1)
  rt0        averaged side fluxes after CP1 (B_1 of CP2), the step's fluxes
             and the RT0 velocity (eq. flux_k_+_2/3, eq. eta_flux; App. A,
             eq. RT0)
  ic0        incomplete Cholesky with no fill, the paper's preconditioner,
             for iteration-count context only (Sec. 3.2.2, 3.2.3)

Parity status: every function above is pinned by tests/test_oracle_*.py
against closed forms, invariants, special cases or brute force; none is
"parity unpinned".
"""
