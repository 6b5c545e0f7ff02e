"""FP64 CPU oracle for SymPix local-operator sampling.

TEST INFRASTRUCTURE ONLY. Nothing on the product path imports, calls or links
anything in this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it. It shares no code with the HIP library
(no kernels, headers, tables or helpers); the only thing both sides consume is
the seeded synthetic input generators in ``workloads``, which hold none of the
method's arithmetic.

Modules
-------
grid       ring latitudes and weights, polar cut, tile-count optimisation,
           pixel layout and tile adjacency (Section 2, Fig. 3, Eqs. 2-5).
kernel     the Legendre-series kernel of Eq. 10, evaluated by direct sum.
operators  pair geometry, the local blocks of D-hat and B-hat (Eq. 16 and
           the tile truncation of Section 4.2), and the blockwise product
           B-hat^T N^-1 B-hat (Eq. 15).
twogrid    B-hat = Y_2 B Y_1^T between an auxiliary grid and the grid of the
           unknowns (Eqs. 13 and 16) and its B-hat^T N_2^-1 B-hat.
sht        spherical harmonic synthesis, its transpose and the quadrature
           analysis of Eq. 1 on the SymPix geometry (real orthonormal basis),
           and the N^-1 degrade theta_2 = W_2 Y_2 Y_obs^T theta of Eq. 14.
precond    the block-Jacobi factor of the system matrix of Section 4.2:
           Cholesky of every tile's diagonal block of D-hat + B-hat^T N^-1
           B-hat, and its solve.
brute      pattern-level brute force without any symmetry reuse (tests only).

Every function is plain and slow on purpose: the point is that a reader can
check it against the paper by eye.
"""
