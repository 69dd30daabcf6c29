"""CPU FP64 oracle for the sparse determinant-ratio VMC hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package.  The
product path (the HIP library and its binding) never calls it and shares no code
with it: the only common dependency is the input generator module
``workloads``, which holds no arithmetic of the method.

Contents (each module cites the part of the paper it follows):

- ``rng``       Philox4x64-10 counter RNG (Salmon et al., SC'11) and the move
                draws of one Metropolis step.
- ``geometry``  minimum image, orbital values, dense Slater matrix, sparsity
                pattern (Section 2.1, eqs. (SlaterMatrix), (gaussian)).
- ``ratio``     determinant ratio by its definition: dense LU solve, brute-force
                Leibniz determinants for tiny n, and the "standard algorithm"
                (explicit inverse with Sherman-Morrison), eqs. (DetRatio),
                (detRatioEq).
- ``reorder``   the geometric greedy particle/orbital reordering (Section 3.1).
- ``ilutp``     threshold ILU with column pivoting, row-wise (Section 3.2,
                eq. (ilu); Section 4 settings).
- ``gmres``     right-preconditioned full GMRES with the effective-stability
                monitor N (eq. (stabilityVecEq)) and the product-form
                preconditioner update (eqs. (mkp1), (finalMkm)).
- ``chain``     Metropolis chain driver: free run and replay of a logged run.

Parity pins: every function here is tied by a ``-m "not gpu"`` test to something
other than itself (a library routine, brute force, a closed form or a
hand-worked example).  Functions without such a pin say so in their docstring.
"""
