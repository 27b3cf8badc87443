"""Plain CPU oracle for the matrix-free DG compressible Navier--Stokes operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything under ``oracle/``; only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.

What it is: a slow, obviously correct, float64 evaluation of the weak form of
Fehn, Wall & Kronbichler (arXiv 1806.03095), Sec. 2.2, eq.
(WeakFormulationConservedVariables), by direct summation over every quadrature
point with dense per-cell basis matrices.  It does no sum factorisation, no
fusion and no reordering beyond what the definition states, so that a reader
can check it against the paper by eye.

Modules
    rules        1D Gauss-Legendre / Gauss-Lobatto rules, Lagrange bases (Sec. 2.2.1, 2.2.3)
    mesh         hexahedral box meshes, isoparametric mapping, geometry (Sec. 2.2.1, 2.2.3, 5.3)
    physics      pointwise fluxes and constitutive laws (Sec. 2.1)
    operator     the DG residual, inverse mass matrix and L(U) (Sec. 2.2.2, 2.2.3, 2.4)
    timeint      explicit low-storage Runge-Kutta and the time-step formula (Sec. 2.4)
    diagnostics  kinetic energy, dissipation, conserved totals (Sec. 5.2.3)
    initial      Taylor-Green and channel initial states, L2 projection (Sec. 5.2.1, 5.3.1)

The state-dependent parts use plain PyTorch CPU ops in float64 so that
reverse-mode automatic differentiation of this definition gives the oracle's
gradient for adjoint checks.
"""

from . import rules, mesh, physics, operator, timeint, diagnostics, initial  # noqa: F401
