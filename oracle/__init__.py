"""Plain FP64 CPU oracle for particle-in-cell current deposition (MatrixPIC, arXiv 2601.08277).

TEST INFRASTRUCTURE ONLY. Nothing on the product path imports this package: only the
tests, the smoke check and the CPU-baseline leg of the benchmark call it. It shares no
code with the HIP library (no kernels, headers, helpers, tables or constant generators).

Contents
--------
shapes   1D B-spline shape factors of order 1..3 on nodal and half-cell (staggered)
         positions, their derivatives, and the continuous kernels B_o(t).
deposit  Eq. 1 of the paper (Sec. 3.1) evaluated directly: per-particle stencil
         scatter, an all-pairs brute-force evaluation, the adjoint (gather) of the
         deposit, the constant-velocity drift used between steps, the field gather,
         the relativistic Boris push and the time-centred (midpoint) current.
esirkepov  The charge-conserving current of Esirkepov's density decomposition (the
         scheme the paper lists as unsupported), from old and new positions.
binning  Cell index of a particle, the cell-sorted binning any correct sorter must
         reproduce (as sets per cell), mover counts, and the global re-sort policy
         of Sec. 4.4.
"""
