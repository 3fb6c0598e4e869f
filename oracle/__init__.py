"""Plain FP64 CPU oracle of the block-preconditioned FSI Jacobian solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never calls it, links it or reads anything it writes at run time, and
this package imports nothing from the GPU library.  Both sides read the same
seeded inputs from ``fsigen`` and nothing else.

What it computes (paper: Jodlbauer, Langer, Wick, "Parallel
Block-Preconditioned Monolithic Solvers for Fluid-Structure-Interaction
Problems"):

* ``blocks``   - the 3x3 block matrix A_h (Section 3.4) and its mat-vec,
                 the solid and fluid sub-blocks and the derived operators
                 (solid Schur matrix, Section 4.3; fluid Schur approximation,
                 Section 4.4 as read in the design notes).
* ``amg``      - smoothed-aggregation AMG setup and V(1,1) Jacobi cycle used
                 for every approximate inverse (Sections 4.2-4.4), dense LU
                 with partial pivoting for the coarsest level.
* ``precond``  - the approximate block-LDU preconditioner application
                 (Algorithm "Evaluation of P^{-1} r", Section 4.1) and the solid
                 Schur-complement algorithm of Section 4.3.
* ``krylov``   - flexible GMRES(m), right preconditioned, modified
                 Gram-Schmidt Arnoldi and Givens least squares.
* ``mlp``      - FP64 reference of the per-node MLP smoother used as a
                 learned replacement for one Jacobi sweep.

Everything here is FP64 and written for clarity, not speed.  Parity status of
each function (what pins it) is listed in its docstring; a function marked
"parity unpinned" has no independent check.
"""
