"""CPU FP64 oracle for accelerated cyclic reduction (ACR).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package;
only the tests, the smoke check and the CPU-baseline leg of the benchmark
call it.  It shares no code with the HIP path: it has its own assembly,
cluster/block trees, H-arithmetic, cyclic reduction and Krylov solvers,
written in plain numpy/scipy for readability, not speed.

Modules
  assembly  -- 7-point operators (variable Poisson with harmonic face
               averages, upwind convection-diffusion, Helmholtz shift)
  dense_cr  -- exact block cyclic reduction with dense plane blocks
  hmatrix   -- cluster tree, block tree, truncation, H-matvec/add/mul/inv
  hacr      -- cyclic reduction with every plane block an H-matrix
  krylov    -- PCG (Fletcher-Reeves / flexible Polak-Ribiere), GMRES(m)
  gradient  -- adjoint gradient of J = 0.5 ||u(kappa) - u_obs||^2
"""
