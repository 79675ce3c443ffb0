"""CPU FP64 oracle for the multiple-Arnoldi Green's-function path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call or
link anything here; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code, constants or helpers with the GPU
path: it rebuilds the tight-binding matrices from atomic positions with its own
Slater-Koster code and follows the method step by step in plain NumPy/SciPy.

Modules
  sk        Slater-Koster carbon sp model: H, S blocks and their derivatives.
  neighbors brute-force minimum-image pair lists, sparsity pattern, clusters.
  fermi     Fermi-Dirac occupation, entropy and bisection for the chemical
            potential.
  krylov    one column of the multiple Arnoldi method (mode K), the dense
            cluster limit (mode D) and the Green's-function column.
  solve     drivers: all columns, chemical potential, density matrix,
            energies, forces, and the whole-system exact reference (mode W).

Modes (readings of the paper, whose letter defers the algorithm to a separate
publication): K follows the Krylov-projection algorithm; D replaces the Krylov
space by the whole cluster (the nu -> n_C limit); W solves the whole system
exactly (dense generalized eigenproblem, dense (zS - H)^-1) for tiny cells.
"""
