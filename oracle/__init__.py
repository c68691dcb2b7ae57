"""CPU oracle for the ADER-AFE-DG hot path (test infrastructure only).

A plain, slow, FP64 numpy implementation of what the method computes, written
from the paper (Michel, Diazzi, Boscheri: continuous 3D finite element subgrid
basis functions for DG on polyhedral meshes).  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
path never does.  It shares no code with the HIP library.

Modules:
    refelem  -- reference tetrahedron: P_N Lagrange basis (App. A), exact
                rational mass/stiffness/derivative/face matrices (Sec. 4.1,
                eqs. for K_xi, V_xi, Z), Gauss-Legendre time basis (Sec. 4.3)
    subgrid  -- sub-tetrahedral split of each polyhedron, agglomerated
                continuous DOFs "without repetition" (Sec. 4.1), sub-tet
                Jacobians, boundary sub-triangles and their neighbour pairing
    physics  -- Navier-Stokes flux, stress tensor, EOS, eigenvalues (Sec. 2)
    scheme   -- CFL time step (Sec. 4.2), detector and artificial viscosity
                (Sec. 4.5), space-time predictor (Sec. 4.3, eq:ader4),
                quadrature-free corrector with Rusanov fluxes (Sec. 4.4)

Every reading taken where the paper is silent or garbled is stated at the
function that takes it.
"""
