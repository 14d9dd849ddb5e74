"""Plain FP64 CPU oracle for the Q^k spectral-element fast-diagonalisation solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code with
the GPU library and never imports it.

Every function follows the paper (Liu, Shen & Zhang, "A simple GPU
implementation of spectral-element methods for solving 3D Poisson type
equations on rectangular domains and its applications", arXiv 2310.00226) and
cites the section / equation it restates.  All arithmetic is float64; numpy's
matmul and symmetric eigensolver serve as library primitives.  The eigenpairs
alone go beyond float64: a long-double cyclic Jacobi iteration (eigjac.c) on the
operator assembled from 40-digit element matrices (mpmath), started from
numpy's eigenvectors, pinned against a 30-digit mpmath reference.

Parity status of each function (what pins it is in tests/test_oracle_*.py):
  gll, diff_matrix, element_matrices, axis_operators, axis_eigen   pinned
  element_matrices_hp (through axis_eigen, 30-digit reference)     pinned
  fd_solve, apply_h3, residual, residual_at, dense_system          pinned
  ch_step                                                          pinned
  schrodinger_apply, pcg_schrodinger                               pinned
    (its iteration counts: pinned at beta = 1 by Table tab7c's 10; parity
     unpinned at beta >= 10, where no reading of the stop reproduces the table)
  spectral_apply                                                   pinned
  periodic boundary condition (axis_operators, axis_eigen, Problem) pinned
  lift_boundary                                                    pinned
  per-axis boundary conditions (Problem with three conditions)     pinned
"""
from .sem_oracle import (  # noqa: F401
    gll,
    legendre,
    diff_matrix,
    element_matrices,
    axis_operators,
    axis_eigen,
    Problem,
    fd_solve,
    mode_product,
    apply_h3,
    residual,
    residual_at,
    dense_system,
    dense_solve,
    ch_step,
    ch_operator_residual,
    schrodinger_apply,
    pcg_schrodinger,
    spectral_apply,
    lift_boundary,
    rel_max_err,
)
