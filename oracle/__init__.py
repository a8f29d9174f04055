"""CPU FP64 oracle for the stage-coupled Vanka multigrid method.

TEST INFRASTRUCTURE ONLY.  Plain, slow, readable NumPy/SciPy code that restates what
the paper computes, used to check the HIP library.  Only the tests, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path never
does.  It shares no code with the HIP library: it re-derives the mesh numbering,
element matrices, stage system, patches, transfers, V-cycle and FGMRES from the
paper on its own.

Modules
  tableau    Butcher tableaux of the IRK families of Sec. 5 (Sec. 2, eq. "general RK").
  fem        Taylor--Hood P2-P1 spaces, quadrature, element matrices, assembly (Sec. 3.1).
  stage      Kronecker stage system and its right-hand side (Sec. 3.1, stage system).
  transfer   Canonical P2 / P1 interpolation between nested meshes (Sec. 4.1).
  vanka      Vertex-star patches and the weighted additive sweep (Sec. 4.2).
  multigrid  Level hierarchy, coarse direct solve and V-cycle (Sec. 4.1, 4.2, 5.1).
  fgmres     Flexible GMRES with right preconditioning (Sec. 4).
  timestep   IRK time stepping, errors, semi-discrete reference solution (Sec. 3.1, 5.1).
  adjoint    Transposed solves and gradients of a tracking loss (not in the paper).
  navier_stokes  Navier--Stokes stage equations, their Jacobian, Newton with
             Eisenstat--Walker forcing (Sec. 3.2).

Pin status of every function is listed in each module header.
"""
