"""FP64 CPU oracle for the space-time Biot slab solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does.

A plain, slow, assembled implementation written from the paper's
definitions (Koecher, "Space-Time-Parallel Poroelasticity Simulation"):
  * `temporal`  -- dG(r) on right Gauss-Radau points (section "Discretisation
                   in Time"), real block form of the temporal matrix
                   (section "Monolithic Approach");
  * `fe`        -- Q2 / RT1 / DG-Q1 element matrices by 3-point Gauss
                   quadrature and global sparse assembly (sections
                   "Poroelasticity", "Discretisation in Space");
  * `slab`      -- the monolithic slab matrix, right-hand side and slab
                   marching with a direct sparse LU (SuperLU) solve;
  * `adjoint`   -- pressure-misfit functional and its discrete-adjoint
                   gradient with respect to cellwise log K;
  * `terzaghi`  -- the 1D consolidation series used as an analytic pin.
Every function is pinned by tests under tests/ (no function is parity
unpinned; see the test files for the pin of each).
"""
