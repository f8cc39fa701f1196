"""Plain FP64 CPU oracle for the w-BFBT Stokes hot path (arXiv 1607.03936).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP library.

Everything here is written from the paper's definitions, in numpy/scipy,
assembled and slow on purpose:

* ``fem``      -- reference element, mesh numbering, assembled A, B, B^T, F,
                  lumped weighted velocity masses (eq. 4, 8, Sec. 5), transfers.
* ``sinker``   -- the multi-sinker viscosity and body force (Sec. 2.1).
* ``solver``   -- Chebyshev-Jacobi smoothing, Lanczos eigenvalue estimate,
                  multigrid V-cycles, the w-BFBT apply (eq. 8), the block
                  preconditioner (eq. 3), flexible GMRES and direct solves.
* ``learned``  -- the small convolutional coarse-correction network.

Parity status per function is listed in each module header.
"""
