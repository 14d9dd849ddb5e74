"""MI355X-native fast-diagonalisation solver for Q^k spectral-element
discretisations of -Lap u + alpha u = f on 3D boxes (arXiv 2310.00226).

The compute path is the HIP library lib/libsemfd.so (C ABI: include/sem.h);
this package is its thin Python binding.
"""
from .binding import (Batch, CahnHilliard, Plan, SemError, axis_fold_host, axis_host, lib,  # noqa: F401
                      PRECISIONS, tune_stats)

__all__ = ["Batch", "CahnHilliard", "Plan", "SemError", "axis_fold_host", "axis_host", "lib", "PRECISIONS",
           "tune_stats"]
