"""CPU FP64 oracle for the finite-temperature Lanczos method (FTLM).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, link or run
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP implementation; the only
common module is the seeded parameter generator ``ftlm_workloads``.

Contents
--------
* :mod:`oracle.dense`  -- textbook spin matrices, the Hamiltonian of Sec. 2.1
  (Heisenberg + single-ion anisotropy + Zeeman + dipolar) built from Kronecker
  products, and exact thermodynamics by full diagonalisation.
* :mod:`oracle.ftlm`   -- FTLM following Sec. 2.2: Gaussian random vectors
  (Eqs. E-1-1, E-1-2), Lanczos recursion, Krylov eigenpairs and the Boltzmann
  sums of Eqs. E-2-C and E-2-D; the heavy H*v and Lanczos loops run in the
  plain C library ``oracle/csrc/ftlm_oracle.c``.
* :mod:`oracle.mlp`    -- FP64 NumPy reference of the surrogate MLP.

Parity status: see the header of each module.
"""
