"""Plain, slow, FP64 CPU oracle of structure-preserving FDTD reduction.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the
product path (the HIP library and its Python binding) never does, and this
package imports nothing from the product path.

Li, Sarris, Triverio, "Structure-Preserving Reduction of Finite-Difference
Time-Domain Equations with Controllable Stability Beyond the CFL Limit"
(arXiv 1406.7042).  Every function cites the section / equation it follows.

Modules
  yee      Sec. II-A: Yee grid, the matrices of eq. (matrix)/(R_and_F), the
           leapfrog of eq. (MNAform), the energy x^T R x; CFL eq. (CFL).
  mor      Sec. II-C, IV-A, IV-B: expansion points eq. (distrib), shifted
           solves, block Arnoldi, SPRIM split eq. (V), projection
           eq. (R_and_Freduced), reduced leapfrog eq. (reducedMNAform).
  perturb  Sec. III-A: singular-value clamp that enforces eq. (singular_limit).
  adjoint  Discrete adjoint of eq. (MNAform) and eq. (reducedMNAform) for
           probe-energy objectives (not in the paper; derived from the same
           equations), plus central finite differences.

Readings of the paper taken where it is silent or garbled are listed in the
design notes of the repository (each one is also stated where it is used).
"""
