"""FP64 CPU oracle for the inverse-DFT hot path — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. The GPU library never calls it, links it or reads its
output at run time, and this package never imports the GPU library.

It computes, by plain and slow means, the discrete quantities of the paper's
finite-element inverse DFT (Sec. 2 and Sec. 3.2):

* ``fe``      — 1-D spectral-element tables (Eq. 12, GLL nodes, Sec. 3.2.1) and the
                3-D standard-form Kohn-Sham operator (Eqs. 17 and 19), both as an
                assembled sparse matrix and as Kronecker-factored 1-D applies.
* ``ks``      — forward eigenproblem (Eq. 19), density (Eq. 4), loss (Eq. 1),
                adjoint right-hand side and solution (Eqs. 7, 10, 20), gradient
                (Eqs. 11, 22), central finite differences.
* ``chfsi``   — the Chebyshev filter polynomial and Rayleigh-Ritz projection
                (Sec. 3.2.2, Eqs. 23-24) by their plain definitions.
* ``vxcmesh`` — the XC potential on its own linear mesh (Eq. 14): the prolongation
                to the orbital nodes and the gradient's transpose (Eq. 22).
* ``hartree`` — the Hartree potential by a finite-element Poisson solve with the
                monopole split off in closed form (the Hamiltonian of Sec. 2).
* ``xcinit``  — the initial guess of Eq. 25 (Slater exchange, PW92 correlation,
                Fermi-Amaldi tail).
* ``mapped``  — smoothly mapped hexahedral meshes: the isoparametric geometry, every
                cell's own dense element stiffness by Gauss quadrature (Eq. 17, Sec. 3.2.3),
                the lumped mass and the standard-form operator on them (Eq. 19).
* ``thermal`` — finite temperature: Fermi-Dirac occupancy and mu (Eqs. 4, 5), the
                adjoint of each degenerate block with Eqs. 8-9 (Sec. 2, Sec. 3.2.2),
                the gradient of Eq. 10.

Every function states the passage it follows. Nothing here is blocked, fused
or reordered beyond what the definition states.
"""
